// mlp.hip -- the residual network of the learned section surrogate on the
// matrix cores of gfx950: forward (inference and training), backward,
// weight gradients and the Adam update.
//
// Network (6 -> 256 -> 256 -> 256 -> 6): h1 = silu(W1 u + b1),
// h2 = h1 + silu(W2 h1 + b2), h3 = h2 + silu(W3 h2 + b3), o = W4 h3 + b4.
// Training runs its matrix products on v_mfma_f32_16x16x32_bf16 and inference
// on v_mfma_f32_32x32x16_bf16 (its tile is described further down); both take
// bfloat16 operands with FP32 accumulation.  Weights enter as bfloat16
// rounded from the FP32 master copy.
// Activations enter either as one bfloat16 (TRK_MLP_BF16) or as the sum of
// two (TRK_MLP_BF16X2: hi = bf16(h), lo = bf16(h - hi), two products into
// one accumulator), which carries 16 significant bits.
//
// Work split (training): a workgroup of four waves owns a tile of 64 rows (particles).
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

#ifndef INFER_NT
#define INFER_NT 2
#endif

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
// Inference evaluates Y^T = W H^T on v_mfma_f32_32x32x16_bf16: the weights are
// the A operand (32 output features x 16 k), the tile's activations the B
// operand (16 k x 32 particles).  Lane l supplies A row / B column l%32 with
// the eight k values 8(l/32)..+7, and receives D rows 8i + 4(l/32) + j
// (i, j = 0..3) of column l%32 in element 4i + j.
//
// Activations sit in LDS in that accumulator order: position
// p = 32b + 16h + 4i + j of a particle's row holds feature 32b + 8i + 4h + j
// (b the 32-feature block, h the lane half).  A lane's sixteen results of a
// block are sixteen consecutive positions (two 16-byte stores per half), the
// next layer reads sixteen consecutive positions per K step, and the input
// columns of the inference weight copies are permuted to match: the same
// sum over k in another order.  At a row stride of 264 bf16 (132 dwords) the
// 16-byte stores and loads of a lane group fall on distinct banks.
//
// Work split: a workgroup of four waves owns 64 particles; wave w computes
// features [64w, 64w + 64) of each hidden layer for all of them (2 x 2
// accumulator blocks).  The skip path keeps each lane's previous activations
// in FP32 registers, as the training forward does; the output layer splits
// K between wave pairs and adds the two halves in a fixed order.  Two
// workgroups share a compute unit (78 KB of LDS each), so the matrix cores of
// one overlap the SiLU epilogue of the other.
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kULds2 = kMlpInK + 8;  // input-tile row stride (bf16)

__device__ __forceinline__ f32x16 mma32(f32x16 c, bf16x8 a, bf16x8 b) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// acc[mt][nt] = W(rows f0 + 32mt .., KS*16 k) x H^T(KS*16 k, particles 32nt ..).
// Software pipelined: the weight fragments (from L2) are loaded three K steps
// ahead and the activation fragments (from LDS) one step ahead, so a step's
// matrix products wait only for data requested two to three steps earlier.
// The first step starts from a zero accumulator operand.
template <int kX2, int KS, int NT>
__device__ __forceinline__ void kloop32(f32x16 (&acc)[2][NT], const uint16_t *__restrict__ w,
                                        int wstride, int f0, const uint16_t *bh,
                                        const uint16_t *bl, int bstride) {
  constexpr int kA = KS < 3 ? KS : 3;  // weight steps in flight
  const int l = threadIdx.x & 63, r = l & 31, h = l >> 5;
  const uint16_t *wr0 = w + static_cast<size_t>(f0 + r) * wstride + 8 * h;
  const uint16_t *wr1 = wr0 + static_cast<size_t>(32) * wstride;
  const uint16_t *b0 = bh + r * bstride + 8 * h;
  const uint16_t *c0 = bl + r * bstride + 8 * h;
  bf16x8 a[kA][2], x[2][NT], y[2][NT];
#pragma unroll
  for (int q = 0; q < kA; ++q) {
    a[q][0] = ld8(wr0 + 16 * q);
    a[q][1] = ld8(wr1 + 16 * q);
  }
#pragma unroll
  for (int nt = 0; nt < NT; ++nt) {
    x[0][nt] = ld8(b0 + 32 * nt * bstride);
    if constexpr (kX2) y[0][nt] = ld8(c0 + 32 * nt * bstride);
  }
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const int cur = s & 1, nxt = cur ^ 1, sa = s % kA;
    // the fences keep the compiler from sinking the early loads next to
    // their use (it does, to save registers, and the wave then stalls on
    // the L2 latency every step)
    __builtin_amdgcn_sched_barrier(0);
    if (s + 1 < KS) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        x[nxt][nt] = ld8(b0 + 32 * nt * bstride + 16 * (s + 1));
        if constexpr (kX2) y[nxt][nt] = ld8(c0 + 32 * nt * bstride + 16 * (s + 1));
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    const f32x16 z = {};
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[mt][nt] = mma32(s == 0 ? z : acc[mt][nt], a[sa][mt], x[cur][nt]);
    if constexpr (kX2) {
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mma32(acc[mt][nt], a[sa][mt], y[cur][nt]);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (s + kA < KS) {
      a[sa][0] = ld8(wr0 + 16 * (s + kA));
      a[sa][1] = ld8(wr1 + 16 * (s + kA));
    }
  }
  __builtin_amdgcn_sched_barrier(0);
}

// bias, SiLU, skip (kFirst: none), the new activations as hi (and lo) bf16
// into the tile at their positions; prev keeps them in FP32
template <int kX2, bool kFirst, int NT>
__device__ __forceinline__ void epi32(const f32x16 (&acc)[2][NT], f32x16 (&prev)[2][NT],
                                      const float *__restrict__ bias, uint16_t *hh, uint16_t *hl,
                                      int f0) {
  const int l = threadIdx.x & 63, r = l & 31, h = l >> 5;
#pragma unroll
  for (int mt = 0; mt < 2; ++mt) {
    float bb[16];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float4 q = *reinterpret_cast<const float4 *>(bias + f0 + 32 * mt + 8 * i + 4 * h);
      bb[4 * i] = q.x;
      bb[4 * i + 1] = q.y;
      bb[4 * i + 2] = q.z;
      bb[4 * i + 3] = q.w;
    }
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      float v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const float s = silu(acc[mt][nt][q] + bb[q]);
        v[q] = kFirst ? s : prev[mt][nt][q] + s;
        prev[mt][nt][q] = v[q];
      }
      uint32_t ph[8], pl[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        ph[t] = pack_bf16(v[2 * t], v[2 * t + 1]);
        if constexpr (kX2) pl[t] = pack_bf16(v[2 * t] - lo_half(ph[t]), v[2 * t + 1] - hi_half(ph[t]));
      }
      const int o = (32 * nt + r) * kLds + f0 + 32 * mt + 16 * h;
      *reinterpret_cast<uint4 *>(hh + o) = uint4{ph[0], ph[1], ph[2], ph[3]};
      *reinterpret_cast<uint4 *>(hh + o + 8) = uint4{ph[4], ph[5], ph[6], ph[7]};
      if constexpr (kX2) {
        *reinterpret_cast<uint4 *>(hl + o) = uint4{pl[0], pl[1], pl[2], pl[3]};
        *reinterpret_cast<uint4 *>(hl + o + 8) = uint4{pl[4], pl[5], pl[6], pl[7]};
      }
    }
  }
}

// Particles per inference workgroup: 32 * kInferNT (each wave holds
// kInferNT 32-particle column tiles of its 64 features)
constexpr int kInferNT = INFER_NT;
constexpr int kIRows = 32 * kInferNT;
constexpr int kOutParts = 4 / kInferNT;  // output layer: K split over the waves
constexpr int kInferWaves = kInferNT == 4 ? 1 : (kInferNT == 2 ? 2 : 3);  // waves per SIMD the LDS allows

// LDS of one inference workgroup
struct InferLds {
  uint16_t hh[kIRows * kLds];
  uint16_t hl[kIRows * kLds];
  uint16_t uh[kIRows * kULds2];
  uint16_t ul[kIRows * kULds2];
  float op[kOutParts][kIRows * 8];  // output-layer K parts
};

// thread t < kIRows: particle t's normalised inputs (s ignored) as hi/lo bf16
__device__ __forceinline__ void put_row(InferLds &L, int t, const float (&u)[kMlpIn]) {
  uint32_t ph[8] = {}, pl[8] = {};
#pragma unroll
  for (int k = 0; k < kMlpIn; k += 2) {
    const float a = k == kMlpSCol ? 0.0f : u[k];
    const float b = k + 1 == kMlpSCol ? 0.0f : u[k + 1];
    ph[k / 2] = pack_bf16(a, b);
    pl[k / 2] = pack_bf16(a - lo_half(ph[k / 2]), b - hi_half(ph[k / 2]));
  }
  uint16_t *uh = L.uh + t * kULds2, *ul = L.ul + t * kULds2;
  *reinterpret_cast<uint4 *>(uh) = uint4{ph[0], ph[1], ph[2], ph[3]};
  *reinterpret_cast<uint4 *>(uh + 8) = uint4{ph[4], ph[5], ph[6], ph[7]};
  *reinterpret_cast<uint4 *>(ul) = uint4{pl[0], pl[1], pl[2], pl[3]};
  *reinterpret_cast<uint4 *>(ul + 8) = uint4{pl[4], pl[5], pl[6], pl[7]};
}

// The network for the kIRows particles whose inputs are in L.uh/L.ul;
// thread t < kIRows reads output k of particle t as out_of(m, L, t, k).
template <int kX2>
__device__ void infer_tile32(const MlpDev &m, InferLds &L) {
  constexpr int NT = kInferNT;
  const int l = threadIdx.x & 63, r = l & 31, h = l >> 5, w = threadIdx.x >> 6, f0 = 64 * w;
  const uint16_t *wi = m.wi;
  f32x16 acc[2][NT], prev[2][NT];
  kloop32<kX2, kMlpInK / 16, NT>(acc, wi, kMlpInK, f0, L.uh, L.ul, kULds2);
  epi32<kX2, true, NT>(acc, prev, m.b1, L.hh, L.hl, f0);
  __syncthreads();
  kloop32<kX2, kMlpHid / 16, NT>(acc, wi + kOffW2i, kMlpHid, f0, L.hh, L.hl, kLds);
  __syncthreads();  // every wave has read h1 before it is overwritten
  epi32<kX2, false, NT>(acc, prev, m.b2, L.hh, L.hl, f0);
  __syncthreads();
  kloop32<kX2, kMlpHid / 16, NT>(acc, wi + kOffW3i, kMlpHid, f0, L.hh, L.hl, kLds);
  __syncthreads();
  epi32<kX2, false, NT>(acc, prev, m.b3, L.hh, L.hl, f0);
  __syncthreads();
  // output layer: wave w takes particles 32(w % NT).. and K part w / NT
  {
    constexpr int kKS = (kMlpHid / 16) / kOutParts;  // K steps per part
    const int nt = w % NT, kp = w / NT;
    const uint16_t *wa = wi + kOffW4i + r * kMlpHid + 8 * h + 16 * kKS * kp;
    const uint16_t *xb = L.hh + (32 * nt + r) * kLds + 8 * h + 16 * kKS * kp;
    const uint16_t *xl = L.hl + (32 * nt + r) * kLds + 8 * h + 16 * kKS * kp;
    f32x16 o = {};
#pragma unroll 2
    for (int s = 0; s < kKS; ++s) {
      const bf16x8 a = ld8(wa + 16 * s);
      o = mma32(o, a, ld8(xb + 16 * s));
      if constexpr (kX2) o = mma32(o, a, ld8(xl + 16 * s));
    }
    // element j (i = 0) holds output 4h + j of particle 32nt + r
    float *op = L.op[kp] + (32 * nt + r) * 8 + 4 * h;
    if (h == 0) {
      op[0] = o[0];
      op[1] = o[1];
      op[2] = o[2];
      op[3] = o[3];
    } else {
      op[0] = o[0];
      op[1] = o[1];
    }
  }
  __syncthreads();
}

__device__ __forceinline__ float out_of(const MlpDev &m, const InferLds &L, int t, int k) {
  float v = L.op[0][t * 8 + k];
#pragma unroll
  for (int q = 1; q < kOutParts; ++q) v += L.op[q][t * 8 + k];
  return v + m.b4[k];
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

// Inference copies of the bfloat16 forward weights: W1 with K = 16, and W2,
// W3, W4 (32 rows, 6 used) with their input columns in the tile's position
// order (position p holds feature 32b + 8i + 4h + j for p = 32b + 16h + 4i + j).
__global__ __launch_bounds__(kBlock) void k_mlp_infer_copy(const MlpDev m) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= kMlpInferElems) return;
  uint16_t v;
  if (i < kOffW2i) {
    v = m.w1f[(i / kMlpInK) * kMlpInPad + i % kMlpInK];
  } else {
    const int64_t j = i < kOffW3i ? i - kOffW2i : (i < kOffW4i ? i - kOffW3i : i - kOffW4i);
    const int row = static_cast<int>(j >> 8), p = static_cast<int>(j & 255);
    const int f = 32 * (p >> 5) + 8 * ((p >> 2) & 3) + 4 * ((p >> 4) & 1) + (p & 3);
    if (i < kOffW3i)
      v = m.w2f[row * kMlpHid + f];
    else if (i < kOffW4i)
      v = m.w3f[row * kMlpHid + f];
    else
      v = row < kMlpOut ? m.w4f[row * kMlpHid + f] : uint16_t{0};
  }
  m.wi[i] = v;
}

// ------------------------------------------------------------------ forward
// o = MLP(u) for rows of u[n][8] (columns 0..5; column 4 ignored) -> out[n][8]
template <int kX2>
__global__ __launch_bounds__(kBlock, kInferWaves) void k_mlp_forward(const MlpDev m, const float *__restrict__ u,
                                                           int64_t n, float *__restrict__ out) {
  __shared__ __attribute__((aligned(16))) InferLds L;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kIRows;
  const int t = threadIdx.x;
  if (t < kIRows) {
    float uu[kMlpIn] = {};
    if (row0 + t < n)
#pragma unroll
      for (int k = 0; k < kMlpIn; ++k) uu[k] = u[(row0 + t) * 8 + k];
    put_row(L, t, uu);
  }
  __syncthreads();
  infer_tile32<kX2>(m, L);
  if (t < kIRows && row0 + t < n) {
#pragma unroll
    for (int k = 0; k < 8; ++k) out[(row0 + t) * 8 + k] = k < kMlpOut ? out_of(m, L, t, k) : 0.0f;
  }
}

// ------------------------------------------------------------------ surrogate
// y = C + R z + D o(N(z)) for the admitted particles adm[0 .. *n_adm), in
// place (x, x', y, y', s; delta unchanged).  Thread t < 64 of a workgroup
// holds particle t of the tile in FP64 from its load to its store.
template <int kX2>
__global__ __launch_bounds__(kBlock, kInferWaves) void k_surr_infer(const MlpDev m, const SurrDev c,
                                                          const BeamPtrs6 b,
                                                          const uint32_t *__restrict__ adm,
                                                          const int64_t *__restrict__ n_adm) {
  __shared__ __attribute__((aligned(16))) InferLds L;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * kIRows;
  const int64_t na = *n_adm;
  if (row0 >= na) return;  // whole workgroup
  const int t = threadIdx.x;
  double z[6];
  int64_t idx = -1;
  if (t < kIRows) {
    float uu[kMlpIn] = {};
    if (row0 + t < na) {
      idx = adm[row0 + t];
#pragma unroll
      for (int k = 0; k < 6; ++k) z[k] = b.z[k][idx];
#pragma unroll
      for (int k = 0; k < kMlpIn; ++k) uu[k] = static_cast<float>(z[k] * c.inv_nw[k]);
    }
    put_row(L, t, uu);
  }
  __syncthreads();
  infer_tile32<kX2>(m, L);
  if (idx >= 0) {
#pragma unroll
    for (int i = 0; i < kMlpDCol; ++i)
      b.z[i][idx] = surr_linear(c, z, i) + c.D[i] * static_cast<double>(out_of(m, L, t, i));
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
// the inference copies follow the forward copies the last Adam step wrote
hipError_t launch_infer_copy(const MlpDev &m, hipStream_t st) {
  const int grid = static_cast<int>((kMlpInferElems + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_mlp_infer_copy, dim3(grid), dim3(kBlock), 0, st, m);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpDev &m, const float *u, int64_t n, float *out, int x2,
                              hipStream_t st) {
  const int64_t grid = (n + kIRows - 1) / kIRows;
  if (grid == 0) return hipSuccess;
  if (hipError_t e = launch_infer_copy(m, st); e != hipSuccess) return e;
  if (x2)
    hipLaunchKernelGGL(k_mlp_forward<1>, dim3(grid), dim3(kBlock), 0, st, m, u, n, out);
  else
    hipLaunchKernelGGL(k_mlp_forward<0>, dim3(grid), dim3(kBlock), 0, st, m, u, n, out);
  return hipGetLastError();
}

hipError_t launch_surr_infer(const MlpDev &m, const SurrDev &c, const BeamPtrs6 &b,
                             const uint32_t *adm, const int64_t *n_adm, int64_t n_total, int x2,
                             hipStream_t st) {
  const int64_t grid = (n_total + kIRows - 1) / kIRows;
  if (grid == 0) return hipSuccess;
  if (hipError_t e = launch_infer_copy(m, st); e != hipSuccess) return e;
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
