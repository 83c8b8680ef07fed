// mlp.hip -- the residual network of the learned section surrogate on the
// matrix cores of gfx950: forward (inference and training), backward,
// weight gradients and the Adam update.
//
// Network (6 -> 256 -> 256 -> 256 -> 6): h1 = silu(W1 u + b1),
// h2 = h1 + silu(W2 h1 + b2), h3 = h2 + silu(W3 h2 + b3), o = W4 h3 + b4.
// Matrix products run on v_mfma_f32_16x16x32_bf16 (bfloat16 operands, FP32
// accumulation).  Weights enter as bfloat16 rounded from the FP32 master copy.
// Activations enter either as one bfloat16 (TRK_MLP_BF16) or as the sum of
// two (TRK_MLP_BF16X2: hi = bf16(h), lo = bf16(h - hi), two products into
// one accumulator), which carries 16 significant bits.
//
// Work split: a workgroup of four waves owns a tile of 64 rows (particles).
// The tile's activations live in LDS, row-major, as the A operand; wave w
// computes output columns [64w, 64w + 64) of every hidden layer for all 64
// rows (4 x 4 MFMA tiles), reading its weight rows straight from L2 as the B
// operand (each row is k-contiguous, so a lane's eight k values are one
// 16-byte load).  The accumulator layout (lane l holds rows 4(l/16)..+3 of
// column l%16) makes the transposed stores of the training path
// (activations [feature][row]) 8- or 16-byte vector stores.
//
// MFMA operand layout used here (16x16x32): lane l supplies A row l%16 and
// B column l%16, each with the eight k values 8(l/16)..8(l/16)+7; the sum
// over k does not depend on how k is distributed as long as A and B agree.
#include <algorithm>

#include "mlp.h"
#include "reduce.h"
#include "surrdev.h"

namespace trk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kRows = 64;                 // rows per workgroup
constexpr int kLds = kMlpHid + 8;         // LDS row stride (bf16 elements)
constexpr int kULds = kMlpInPad + 8;      // LDS row stride of the input tile

__device__ __forceinline__ uint16_t bf16_bits(float x) {  // nearest, ties to even
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float bf16_float(uint16_t b) {
  return __uint_as_float(static_cast<uint32_t>(b) << 16);
}

// two floats to two bfloat16 (nearest even) packed low-first, one
// v_cvt_pk_bf16_f32
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
  const bf16x2v v = {static_cast<__bf16>(a), static_cast<__bf16>(b)};
  return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ float lo_half(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi_half(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

__device__ __forceinline__ bf16x8 ld8(const uint16_t *p) {
  return *reinterpret_cast<const bf16x8 *>(p);
}

__device__ __forceinline__ f32x4 mma(f32x4 c, bf16x8 a, bf16x8 b) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// sigma(a) = 1 / (1 + 2^(-a log2 e)) with the hardware exp2 and reciprocal
// (about 1 ulp each; a large negative a gives exp2 = inf and sigma = 0)
__device__ __forceinline__ float sigmoid(float a) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(a * -1.4426950408889634f));
}
__device__ __forceinline__ float silu(float a) { return a * sigmoid(a); }
__device__ __forceinline__ float dsilu(float a) {
  const float s = sigmoid(a);
  return s * (1.0f + a * (1.0f - s));
}

// acc[rt][ct] += A(rows 16rt.., K) * W(rows n0+16ct.., K)^T
template <int kX2, int K>
__device__ __forceinline__ void mma_block(f32x4 (&acc)[4][4], const uint16_t *ah, const uint16_t *al,
                                          int astride, const uint16_t *__restrict__ w, int wstride,
                                          int n0) {
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
#pragma unroll 2
  for (int kk = 0; kk < K / 32; ++kk) {
    bf16x8 b[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
      b[ct] = ld8(w + static_cast<size_t>(n0 + 16 * ct + r) * wstride + 32 * kk + 8 * g);
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const bf16x8 a = ld8(ah + (16 * rt + r) * astride + 32 * kk + 8 * g);
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = mma(acc[rt][ct], a, b[ct]);
      if constexpr (kX2) {
        const bf16x8 a2 = ld8(al + (16 * rt + r) * astride + 32 * kk + 8 * g);
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = mma(acc[rt][ct], a2, b[ct]);
      }
    }
  }
}

__device__ __forceinline__ void zero(f32x4 (&acc)[4][4]) {
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) acc[rt][ct] = f32x4{0.f, 0.f, 0.f, 0.f};
}

// Transposed stores of the training path (feature-major [feature][batch]).
struct Save {
  float *aT[3];
  uint16_t *hT[3];
  int64_t ld;   // batch stride
  int64_t b0;   // batch row of the tile's first row
};

// Epilogue of a hidden layer: bias, SiLU, skip, the new activations into LDS
// (hi/lo) and, when training, the pre-activations and activations to HBM.
template <int kX2, bool kSave>
__device__ __forceinline__ void hidden_epilogue(f32x4 (&acc)[4][4], f32x4 (&h)[4][4], bool first,
                                                const float *__restrict__ bias, uint16_t *hh,
                                                uint16_t *hl, const Save &sv, int layer) {
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4, n0 = 64 * (threadIdx.x >> 6);
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int col = n0 + 16 * ct + r;
    const float bb = bias[col];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      f32x4 a;
      uint16_t hb[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = acc[rt][ct][q] + bb;
        const float s = silu(a[q]);
        const float v = first ? s : h[rt][ct][q] + s;
        h[rt][ct][q] = v;
        const uint16_t hi = bf16_bits(v);
        hb[q] = hi;
        const int row = 16 * rt + 4 * g + q;
        hh[row * kLds + col] = hi;
        if constexpr (kX2) hl[row * kLds + col] = bf16_bits(v - bf16_float(hi));
      }
      if constexpr (kSave) {
        const int64_t o = static_cast<int64_t>(col) * sv.ld + sv.b0 + 16 * rt + 4 * g;
        *reinterpret_cast<f32x4 *>(sv.aT[layer] + o) = a;
        uint2 pk;
        pk.x = static_cast<uint32_t>(hb[0]) | (static_cast<uint32_t>(hb[1]) << 16);
        pk.y = static_cast<uint32_t>(hb[2]) | (static_cast<uint32_t>(hb[3]) << 16);
        *reinterpret_cast<uint2 *>(sv.hT[layer] + o) = pk;
      }
    }
  }
}

// The whole network for one tile whose inputs are in LDS (uh/ul, aliased
// with hh/hl); leaves o[row][0..8) in os (columns >= 6 are zero).
template <int kX2, bool kSave>
__device__ void mlp_tile(const MlpDev &m, uint16_t *hh, uint16_t *hl, float *os, const Save &sv) {
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4, w = threadIdx.x >> 6, n0 = 64 * w;
  f32x4 acc[4][4], h[4][4];
  // layer 1 (K = 32, inputs zero-padded)
  zero(acc);
  mma_block<kX2, kMlpInPad>(acc, hh, hl, kULds, m.w1f, kMlpInPad, n0);
  __syncthreads();  // inputs read by every wave before the tile is overwritten
  hidden_epilogue<kX2, kSave>(acc, h, true, m.b1, hh, hl, sv, 0);
  __syncthreads();
  // layers 2 and 3
  zero(acc);
  mma_block<kX2, kMlpHid>(acc, hh, hl, kLds, m.w2f, kMlpHid, n0);
  __syncthreads();
  hidden_epilogue<kX2, kSave>(acc, h, false, m.b2, hh, hl, sv, 1);
  __syncthreads();
  zero(acc);
  mma_block<kX2, kMlpHid>(acc, hh, hl, kLds, m.w3f, kMlpHid, n0);
  __syncthreads();
  hidden_epilogue<kX2, kSave>(acc, h, false, m.b3, hh, hl, sv, 2);
  __syncthreads();
  // output layer: wave w takes rows 16w..16w+15, one 16-column tile
  f32x4 o{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int kk = 0; kk < kMlpHid / 32; ++kk) {
    const bf16x8 b = ld8(m.w4f + r * kMlpHid + 32 * kk + 8 * g);
    o = mma(o, ld8(hh + (16 * w + r) * kLds + 32 * kk + 8 * g), b);
    if constexpr (kX2) o = mma(o, ld8(hl + (16 * w + r) * kLds + 32 * kk + 8 * g), b);
  }
  if (r < 8) {
#pragma unroll
    for (int q = 0; q < 4; ++q) os[(16 * w + 4 * g + q) * 8 + r] = r < kMlpOut ? o[q] + m.b4[r] : 0.0f;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ inference tile
// Inference evaluates Y^T = W H^T: the weights are the A operand (rows =
// output features, read from L2 one K step ahead of their use), the tile's
// activations the B operand.  The accumulator of lane l then holds four
// consecutive features 4(l/16).. of particle l%16, so the epilogue writes
// each lane's four new activations with one 8-byte LDS store per half.  The
// skip path reads the previous activation back as hi + lo (16 significant
// bits) instead of keeping it in registers, which halves the register
// footprint and lets two workgroups share a compute unit.
template <int kX2, int K>
__device__ __forceinline__ void mma_t(f32x4 (&acc)[4][4], const uint16_t *__restrict__ w, int wstride,
                                      int f0, const uint16_t *bh, const uint16_t *bl, int bstride) {
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
  bf16x8 a[4];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) a[mt] = ld8(w + static_cast<size_t>(f0 + 16 * mt + r) * wstride + 8 * g);
#pragma unroll 1
  for (int kk = 0; kk < K / 32; ++kk) {
    bf16x8 an[4];
    if (kk + 1 < K / 32) {
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
        an[mt] = ld8(w + static_cast<size_t>(f0 + 16 * mt + r) * wstride + 32 * (kk + 1) + 8 * g);
    }
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const bf16x8 b = ld8(bh + (16 * nt + r) * bstride + 32 * kk + 8 * g);
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) acc[mt][nt] = mma(acc[mt][nt], a[mt], b);
      if constexpr (kX2) {
        const bf16x8 b2 = ld8(bl + (16 * nt + r) * bstride + 32 * kk + 8 * g);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) acc[mt][nt] = mma(acc[mt][nt], a[mt], b2);
      }
    }
    if (kk + 1 < K / 32) {
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) a[mt] = an[mt];
    }
  }
}

template <bool kFirst>
__device__ __forceinline__ void epi_t(const f32x4 (&acc)[4][4], const float *__restrict__ bias,
                                      uint16_t *hh, uint16_t *hl, int f0) {
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
    const int f = f0 + 16 * mt + 4 * g;
    float bb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) bb[q] = bias[f + q];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
      const int o = (16 * nt + r) * kLds + f;
      float v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) v[q] = silu(acc[mt][nt][q] + bb[q]);
      if constexpr (!kFirst) {
        const uint2 oh = *reinterpret_cast<const uint2 *>(hh + o);
        const uint2 ol = *reinterpret_cast<const uint2 *>(hl + o);
        v[0] = (lo_half(oh.x) + lo_half(ol.x)) + v[0];
        v[1] = (hi_half(oh.x) + hi_half(ol.x)) + v[1];
        v[2] = (lo_half(oh.y) + lo_half(ol.y)) + v[2];
        v[3] = (hi_half(oh.y) + hi_half(ol.y)) + v[3];
      }
      uint2 ph, pl;
      ph.x = pack_bf16(v[0], v[1]);
      ph.y = pack_bf16(v[2], v[3]);
      pl.x = pack_bf16(v[0] - lo_half(ph.x), v[1] - hi_half(ph.x));
      pl.y = pack_bf16(v[2] - lo_half(ph.y), v[3] - hi_half(ph.y));
      *reinterpret_cast<uint2 *>(hh + o) = ph;
      *reinterpret_cast<uint2 *>(hl + o) = pl;
    }
  }
}

// The network for one 64-particle tile whose inputs are in LDS (uh/ul,
// aliased with hh/hl); leaves o[row][0..8) in os (columns >= 6 zero).
template <int kX2>
__device__ void infer_tile(const MlpDev &m, uint16_t *hh, uint16_t *hl, float *os) {
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4, w = threadIdx.x >> 6, f0 = 64 * w;
  f32x4 acc[4][4];
  zero(acc);
  mma_t<kX2, kMlpInPad>(acc, m.w1f, kMlpInPad, f0, hh, hl, kULds);
  __syncthreads();
  epi_t<true>(acc, m.b1, hh, hl, f0);
  __syncthreads();
  zero(acc);
  mma_t<kX2, kMlpHid>(acc, m.w2f, kMlpHid, f0, hh, hl, kLds);
  __syncthreads();
  epi_t<false>(acc, m.b2, hh, hl, f0);
  __syncthreads();
  zero(acc);
  mma_t<kX2, kMlpHid>(acc, m.w3f, kMlpHid, f0, hh, hl, kLds);
  __syncthreads();
  epi_t<false>(acc, m.b3, hh, hl, f0);
  __syncthreads();
  // output layer: 16 output rows (6 used) x particles 16w..16w+15
  f32x4 o{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int kk = 0; kk < kMlpHid / 32; ++kk) {
    const bf16x8 a = ld8(m.w4f + r * kMlpHid + 32 * kk + 8 * g);
    o = mma(o, a, ld8(hh + (16 * w + r) * kLds + 32 * kk + 8 * g));
    if constexpr (kX2) o = mma(o, a, ld8(hl + (16 * w + r) * kLds + 32 * kk + 8 * g));
  }
  if (g < 2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int out = 4 * g + q;
      os[(16 * w + r) * 8 + out] = out < kMlpOut ? o[q] + m.b4[out] : 0.0f;
    }
  }
  __syncthreads();
}

// input tile: 64 rows x 32 (6 used, s column zero) as hi/lo bf16
__device__ __forceinline__ void put_input(uint16_t *uh, uint16_t *ul, int row, int k, float v) {
  const uint16_t hi = bf16_bits(v);
  uh[row * kULds + k] = hi;
  ul[row * kULds + k] = bf16_bits(v - bf16_float(hi));
}

__device__ __forceinline__ void clear_input(uint16_t *uh, uint16_t *ul) {
  for (int i = threadIdx.x; i < kRows * kULds; i += kBlock) {
    uh[i] = 0;
    ul[i] = 0;
  }
}

}  // namespace

// ------------------------------------------------------------------ forward
// o = MLP(u) for rows of u[n][8] (columns 0..5; column 4 ignored) -> out[n][8]
template <int kX2>
__global__ __launch_bounds__(kBlock) void k_mlp_forward(const MlpDev m, const float *__restrict__ u,
                                                        int64_t n, float *__restrict__ out) {
  __shared__ __attribute__((aligned(16))) uint16_t hh[kRows * kLds];
  __shared__ __attribute__((aligned(16))) uint16_t hl[kRows * kLds];
  __shared__ float os[kRows * 8];
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kRows;
  clear_input(hh, hl);
  __syncthreads();
  for (int i = threadIdx.x; i < kRows * kMlpIn; i += kBlock) {
    const int row = i / kMlpIn, k = i % kMlpIn;
    if (row0 + row < n && k != kMlpSCol) put_input(hh, hl, row, k, u[(row0 + row) * 8 + k]);
  }
  __syncthreads();
  infer_tile<kX2>(m, hh, hl, os);
  for (int i = threadIdx.x; i < kRows * 8; i += kBlock) {
    const int row = i / 8;
    if (row0 + row < n) out[row0 * 8 + i] = os[i];
  }
}


// ------------------------------------------------------------------ surrogate
// y = C + R z + D o(N(z)) for the admitted particles adm[0 .. *n_adm), in
// place (x, x', y, y', s; delta unchanged).  Thread t < 64 of a workgroup
// holds particle t of the tile in FP64 from its load to its store.
template <int kX2>
__global__ __launch_bounds__(kBlock) void k_surr_infer(const MlpDev m, const SurrDev c, const BeamPtrs6 b,
                                                       const uint32_t *__restrict__ adm,
                                                       const int64_t *__restrict__ n_adm) {
  __shared__ __attribute__((aligned(16))) uint16_t hh[kRows * kLds];
  __shared__ __attribute__((aligned(16))) uint16_t hl[kRows * kLds];
  __shared__ float os[kRows * 8];
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kRows;
  const int64_t na = *n_adm;
  if (row0 >= na) return;  // whole workgroup
  clear_input(hh, hl);
  __syncthreads();
  double z[6];
  int64_t idx = -1;
  if (threadIdx.x < kRows && row0 + threadIdx.x < na) {
    idx = adm[row0 + threadIdx.x];
#pragma unroll
    for (int k = 0; k < 6; ++k) z[k] = b.z[k][idx];
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (k != kMlpSCol) put_input(hh, hl, threadIdx.x, k, static_cast<float>(z[k] * c.inv_nw[k]));
  }
  __syncthreads();
  infer_tile<kX2>(m, hh, hl, os);
  if (idx >= 0) {
#pragma unroll
    for (int i = 0; i < kMlpDCol; ++i)
      b.z[i][idx] = surr_linear(c, z, i) + c.D[i] * static_cast<double>(os[threadIdx.x * 8 + i]);
  }
}

// ------------------------------------------------------------------ training
// Forward of one batch with the saves of the backward pass, the targets
// t = r * inv_scale, the loss partial of the tile and dO = (2/(6B)) (o - t).
// Batch row b reads pair (a b_glob + c) mod n_pairs, b_glob = row0 + b.
template <int kX2>
__global__ __launch_bounds__(kBlock) void k_mlp_train_fwd(const MlpDev m, const TrainArgs t) {
  __shared__ __attribute__((aligned(16))) uint16_t hh[kRows * kLds];
  __shared__ __attribute__((aligned(16))) uint16_t hl[kRows * kLds];
  __shared__ float os[kRows * 8];
  __shared__ float ts[kRows * 8];
  __shared__ float lsum[kWaves];
  const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kRows;
  clear_input(hh, hl);
  __syncthreads();
  for (int i = threadIdx.x; i < kRows * 8; i += kBlock) {
    const int row = i / 8, k = i % 8;
    const uint64_t gidx = static_cast<uint64_t>(t.row0 + b0 + row);
    const int64_t p = static_cast<int64_t>((t.perm_a * gidx + t.perm_c) % static_cast<uint64_t>(t.n_pairs));
    if (k < kMlpIn) {
      const float v = k == kMlpSCol ? 0.0f : t.u[p * 8 + k];
      if (k != kMlpSCol) put_input(hh, hl, row, k, v);
      t.uT[static_cast<int64_t>(k) * t.B + b0 + row] = bf16_bits(v);
      ts[i] = t.r[p * 8 + k] * t.inv_scale[k];
    } else {
      ts[i] = 0.0f;
    }
  }
  __syncthreads();
  Save sv;
  for (int k = 0; k < 3; ++k) {
    sv.aT[k] = t.aT[k];
    sv.hT[k] = t.hT[k];
  }
  sv.ld = t.B;
  sv.b0 = b0;
  mlp_tile<kX2, true>(m, hh, hl, os, sv);
  // dO (row-major [B][32] and transposed [16][B]) and the squared error
  const float scale = 2.0f / (6.0f * static_cast<float>(t.B));
  float se = 0.0f;
  for (int i = threadIdx.x; i < kRows * 16; i += kBlock) {
    const int row = i / 16, k = i % 16;
    float d = 0.0f;
    if (k < kMlpOut) {
      d = os[row * 8 + k] - ts[row * 8 + k];
      se += d * d;
    }
    const uint16_t db = bf16_bits(d * scale);
    t.dO[(b0 + row) * kMlpInPad + k] = db;
    t.dOT[static_cast<int64_t>(k) * t.B + b0 + row] = db;
  }
  for (int mm = 32; mm >= 1; mm >>= 1) se += __shfl_xor(se, mm, 64);
  if ((threadIdx.x & 63) == 0) lsum[threadIdx.x >> 6] = se;
  __syncthreads();
  if (threadIdx.x == 0) t.loss_part[blockIdx.x] = ((lsum[0] + lsum[1]) + lsum[2]) + lsum[3];
}

// Backward of one batch: dh3 = dO W4; for layers 3, 2, 1: dA = dh * silu'(a)
// (stored transposed for the weight gradients), dh <- dh + dA W (layers 3, 2).
__global__ __launch_bounds__(kBlock) void k_mlp_train_bwd(const MlpDev m, const TrainArgs t) {
  __shared__ __attribute__((aligned(16))) uint16_t gs[kRows * kLds];
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4, n0 = 64 * (threadIdx.x >> 6);
  const int64_t b0 = static_cast<int64_t>(blockIdx.x) * kRows;
  f32x4 dh[4][4], acc[4][4];
  zero(dh);
  {
    bf16x8 b[4];
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) b[ct] = ld8(m.w4b + (n0 + 16 * ct + r) * kMlpInPad + 8 * g);
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const bf16x8 a = ld8(t.dO + (b0 + 16 * rt + r) * kMlpInPad + 8 * g);
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) dh[rt][ct] = mma(dh[rt][ct], a, b[ct]);
    }
  }
  for (int layer = 2; layer >= 0; --layer) {
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const int col = n0 + 16 * ct + r;
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        const int64_t o = static_cast<int64_t>(col) * t.B + b0 + 16 * rt + 4 * g;
        const f32x4 a = *reinterpret_cast<const f32x4 *>(t.aT[layer] + o);
        uint16_t db[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float d = dh[rt][ct][q] * dsilu(a[q]);
          db[q] = bf16_bits(d);
          if (layer > 0) gs[(16 * rt + 4 * g + q) * kLds + col] = db[q];
        }
        uint2 pk;
        pk.x = static_cast<uint32_t>(db[0]) | (static_cast<uint32_t>(db[1]) << 16);
        pk.y = static_cast<uint32_t>(db[2]) | (static_cast<uint32_t>(db[3]) << 16);
        *reinterpret_cast<uint2 *>(t.dAT[layer] + o) = pk;
      }
    }
    if (layer == 0) break;
    __syncthreads();
    zero(acc);
    mma_block<0, kMlpHid>(acc, gs, gs, kLds, layer == 2 ? m.w3b : m.w2b, kMlpHid, n0);
    __syncthreads();  // every wave has read gs before the next layer rewrites it
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) dh[rt][ct] += acc[rt][ct];
  }
}

// Weight and bias gradients as split-K partials: out[s][M][N] = sum over the
// batch slice s of A[M][.] B[N][.]^T, both operands feature-major bf16.  The
// B operands carry a row of ones after the activations, so the bias
// gradients come out as one more column.  One wave per 16x16 output tile.
__global__ __launch_bounds__(kBlock) void k_mlp_wgrad(const WgradArgs w) {
  const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
  const int64_t gw = static_cast<int64_t>(blockIdx.x) * kWaves + (threadIdx.x >> 6);
  const int64_t s = gw / w.tiles;
  if (s >= w.slices) return;
  int t = static_cast<int>(gw % w.tiles);
  int j = 0;
  while (j < 3 && t >= w.job[j].ntiles) {
    t -= w.job[j].ntiles;
    ++j;
  }
  const WgradJob &J = w.job[j];
  const int mt = t / J.nt, nt = t % J.nt;
  const int64_t k0 = s * w.kslice;
  const uint16_t *pa = J.a + static_cast<int64_t>(16 * mt + r) * w.ld + k0 + 8 * g;
  const uint16_t *pb = J.b + static_cast<int64_t>(16 * nt + r) * w.ld + k0 + 8 * g;
  f32x4 acc{0.f, 0.f, 0.f, 0.f};
  for (int64_t kk = 0; kk < w.kslice; kk += 32) acc = mma(acc, ld8(pa + kk), ld8(pb + kk));
  const int ncol = 16 * J.nt;
  float *o = J.out + (s * 16 * J.mt + 16 * mt + 4 * g) * static_cast<int64_t>(ncol) + 16 * nt + r;
#pragma unroll
  for (int q = 0; q < 4; ++q) o[q * ncol] = acc[q];
}

// ------------------------------------------------------------------ Adam
// One thread per parameter.  mode 0: gradient = sum of the split-K partials,
// then Adam; mode 1: gradient given, then Adam; mode 2: partials summed into
// grad_out only; mode 3: refresh the bf16 copies only.  Adam in binary64 on
// binary32 state (w, m, v), then the bf16 weight copies in both layouts.
__global__ __launch_bounds__(kBlock) void k_mlp_adam(const AdamArgs a) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (a.loss_part != nullptr && blockIdx.x == 0 && threadIdx.x == 0) {
    float s = 0.0f;
    for (int i = 0; i < a.nloss; ++i) s += a.loss_part[i];
    *a.loss_acc = (a.loss_reset ? 0.0f : *a.loss_acc) + s * a.loss_scale;
  }
  if (p >= kMlpNParam) return;
  // (layer, row j, column i) of the parameter; bias = column `bias_col`
  int layer, j, i;
  if (p < kOffB1) { layer = 0; j = static_cast<int>(p / kMlpIn); i = static_cast<int>(p % kMlpIn); }
  else if (p < kOffW2) { layer = 0; j = static_cast<int>(p - kOffB1); i = -1; }
  else if (p < kOffB2) { layer = 1; j = static_cast<int>((p - kOffW2) / kMlpHid); i = static_cast<int>((p - kOffW2) % kMlpHid); }
  else if (p < kOffW3) { layer = 1; j = static_cast<int>(p - kOffB2); i = -1; }
  else if (p < kOffB3) { layer = 2; j = static_cast<int>((p - kOffW3) / kMlpHid); i = static_cast<int>((p - kOffW3) % kMlpHid); }
  else if (p < kOffW4) { layer = 2; j = static_cast<int>(p - kOffB3); i = -1; }
  else if (p < kOffB4) { layer = 3; j = static_cast<int>((p - kOffW4) / kMlpHid); i = static_cast<int>((p - kOffW4) % kMlpHid); }
  else { layer = 3; j = static_cast<int>(p - kOffB4); i = -1; }
  if (a.mode != 3) {
    float g32;
    if (a.mode == 1) {
      g32 = a.grad_in[p];
    } else {
      const int ncol = layer == 0 ? kMlpInPadT : kMlpHT;
      const int nrow = layer == 3 ? kMlpOutPad : kMlpHid;
      const int c = i < 0 ? (layer == 0 ? kMlpIn : kMlpHid) : i;
      const float *part = a.part[layer] + static_cast<int64_t>(j) * ncol + c;
      const int64_t stride = static_cast<int64_t>(nrow) * ncol;
      double gs = 0.0;
      for (int s = 0; s < a.slices; ++s) gs += static_cast<double>(part[s * stride]);
      g32 = static_cast<float>(gs);
    }
    if (a.mode == 2) {
      a.grad_out[p] = g32;
      return;
    }
    const double g = static_cast<double>(g32);
    const double mm = a.b1 * static_cast<double>(a.m[p]) + a.omb1 * g;
    const double vv = a.b2 * static_cast<double>(a.v[p]) + a.omb2 * (g * g);
    const double upd = (a.lr * (mm / a.bc1)) / (sqrt(vv / a.bc2) + a.eps);
    const float wn = static_cast<float>(static_cast<double>(a.w[p]) - upd);
    a.w[p] = wn;
    a.m[p] = static_cast<float>(mm);
    a.v[p] = static_cast<float>(vv);
  }
  if (i < 0) return;  // biases are read in FP32
  const uint16_t b = bf16_bits(a.w[p]);
  switch (layer) {
    case 0: a.w1f[j * kMlpInPad + i] = b; break;
    case 1: a.w2f[j * kMlpHid + i] = b; a.w2b[i * kMlpHid + j] = b; break;
    case 2: a.w3f[j * kMlpHid + i] = b; a.w3b[i * kMlpHid + j] = b; break;
    default: a.w4f[j * kMlpHid + i] = b; a.w4b[i * kMlpInPad + j] = b; break;
  }
}

// fill a bf16 (or any 16-bit) buffer with a constant
__global__ void k_fill_u16(uint16_t *p, int64_t n, uint16_t v) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

// ------------------------------------------------------------------ launchers
hipError_t launch_mlp_forward(const MlpDev &m, const float *u, int64_t n, float *out, int x2,
                              hipStream_t st) {
  const int64_t grid = (n + kRows - 1) / kRows;
  if (grid == 0) return hipSuccess;
  if (x2)
    hipLaunchKernelGGL(k_mlp_forward<1>, dim3(grid), dim3(kBlock), 0, st, m, u, n, out);
  else
    hipLaunchKernelGGL(k_mlp_forward<0>, dim3(grid), dim3(kBlock), 0, st, m, u, n, out);
  return hipGetLastError();
}

hipError_t launch_surr_infer(const MlpDev &m, const SurrDev &c, const BeamPtrs6 &b,
                             const uint32_t *adm, const int64_t *n_adm, int64_t n_total, int x2,
                             hipStream_t st) {
  const int64_t grid = (n_total + kRows - 1) / kRows;
  if (grid == 0) return hipSuccess;
  if (x2)
    TRK_LAUNCH((k_surr_infer<1>), dim3(grid), dim3(kBlock), 0, st, m, c, b, adm, n_adm);
  else
    TRK_LAUNCH((k_surr_infer<0>), dim3(grid), dim3(kBlock), 0, st, m, c, b, adm, n_adm);
  return hipGetLastError();
}

hipError_t launch_mlp_train_fwd(const MlpDev &m, const TrainArgs &t, int x2, hipStream_t st) {
  const int grid = static_cast<int>(t.B / kRows);
  if (x2)
    hipLaunchKernelGGL(k_mlp_train_fwd<1>, dim3(grid), dim3(kBlock), 0, st, m, t);
  else
    hipLaunchKernelGGL(k_mlp_train_fwd<0>, dim3(grid), dim3(kBlock), 0, st, m, t);
  return hipGetLastError();
}

hipError_t launch_mlp_train_bwd(const MlpDev &m, const TrainArgs &t, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_train_bwd, dim3(static_cast<int>(t.B / kRows)), dim3(kBlock), 0, st, m, t);
  return hipGetLastError();
}

hipError_t launch_mlp_wgrad(const WgradArgs &w, hipStream_t st) {
  const int64_t waves = static_cast<int64_t>(w.tiles) * w.slices;
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(static_cast<int>((waves + kWaves - 1) / kWaves)), dim3(kBlock),
                     0, st, w);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(const AdamArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpNParam + kBlock - 1) / kBlock), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fill_u16(uint16_t *p, int64_t n, uint16_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t grid = std::min<int64_t>((n + kBlock - 1) / kBlock, 4096);
  hipLaunchKernelGGL(k_fill_u16, dim3(static_cast<int>(grid)), dim3(kBlock), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace trk
