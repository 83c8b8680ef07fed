// devmath.h -- device arithmetic of the tracker: own elementary functions,
// Philox4x32-10 and the Box-Muller normal.
//
// Every function here has a fixed evaluation order (explicit fma, no
// contraction: the library is built with -ffp-contract=off) so that a CPU
// implementation of the same recipe reproduces it bit for bit:
//   sin/cos  Cody-Waite reduction by pi/2 in three parts (33+33+53 bits),
//            then Taylor polynomials on |r| <= pi/4 (degree 17 / 18) with
//            coefficients (-1)^k / n!, each the correctly rounded 1/n!.
//   log      x = m 2^e, m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(f),
//            f = (m-1)/(m+1), odd series to f^23; e ln2 in two parts.
//   exp      x = k ln2 + r, Taylor to degree 14, times 2^k; 0 below -700.
//   Philox   Salmon, Moraes, Dror & Shaw, SC'11: 10 rounds, multipliers
//            0xD2511F53 / 0xCD9E8D57, key increments 0x9E3779B9 / 0xBB67AE85.
//   normal   53-bit uniforms u1 in (0,1], u2 in [0,1) from the four output
//            words; g = sqrt(-2 log u1) cos(2 pi u2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace trk {
namespace dm {

// 1/n! for n = 0..18, each the correctly rounded quotient of 1 by the exact
// binary64 value of n! (n! is representable for n <= 22).
__device__ __forceinline__ constexpr double inv_fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f = f * static_cast<double>(i);
  return 1.0 / f;
}

constexpr double kPio2Hi = 0x1.921fb54400000p+0;
constexpr double kPio2Mid = 0x1.0b4611a600000p-34;
constexpr double kPio2Lo = 0x1.3198a2e037073p-69;
constexpr double kTwoOverPi = 0x1.45f306dc9c883p-1;
constexpr double kLn2Hi = 0x1.62e42ff000000p-1;
constexpr double kLn2Lo = -0x1.718432a1b0e26p-35;
constexpr double kInvLn2 = 0x1.71547652b82fep+0;
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;
constexpr double kTwoPi = 0x1.921fb54442d18p+2;

// a*b + c rounded once, as one three-address v_fma_f64.  For a Horner step
// whose addend c is a constant held in a register, the compiler's own
// two-address form (v_fmac) first copies the constant into the destination:
// one extra 64-bit move per step.
__device__ __forceinline__ double fma3(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
  return r;
}

// Taylor kernels on the reduced argument.  Horner from the highest degree:
// p <- fma(p, r^2, c_next); sin = fma(r^3, p, r), cos = fma(r^2, p, 1).
__device__ __forceinline__ double sin_kernel(double r) {
  const double r2 = r * r;
  double p = inv_fact(17);
#pragma unroll
  for (int n = 15; n >= 3; n -= 2) {
    const double c = ((n >> 1) & 1) ? -inv_fact(n) : inv_fact(n);
    p = fma3(p, r2, c);
  }
  return fma(r * r2, p, r);
}
__device__ __forceinline__ double cos_kernel(double r) {
  const double r2 = r * r;
  double p = -inv_fact(18);
#pragma unroll
  for (int n = 16; n >= 2; n -= 2) {
    const double c = ((n >> 1) & 1) ? -inv_fact(n) : inv_fact(n);
    p = fma3(p, r2, c);
  }
  return fma(r2, p, 1.0);
}

// |x| < 2^31 pi/2: the quadrant count fits an int
__device__ __forceinline__ double reduce_half_pi(double x, int &q) {
  const double k = __builtin_rint(x * kTwoOverPi);
  const double r = ((x - k * kPio2Hi) - k * kPio2Mid) - k * kPio2Lo;
  q = static_cast<int>(k) & 3;
  return r;
}

__device__ __forceinline__ double own_sin(double x) {
  int q;
  const double r = reduce_half_pi(x, q);
  const double v = (q & 1) ? cos_kernel(r) : sin_kernel(r);
  return (q & 2) ? -v : v;
}
__device__ __forceinline__ double own_cos(double x) {
  int q;
  const double r = reduce_half_pi(x, q);
  const double v = (q & 1) ? sin_kernel(r) : cos_kernel(r);
  return ((q + 1) & 2) ? -v : v;
}

// sin and cos of one argument from one reduction (the same values as own_sin
// and own_cos).  For |x| <= 0.78 < pi/4 the reduction is the identity
// (k = rint(2x/pi) = 0, r = x exactly), so the kernels take x directly.
__device__ __forceinline__ void own_sincos(double x, double &sn, double &cs) {
  if (fabs(x) <= 0.78) {
    sn = sin_kernel(x);
    cs = cos_kernel(x);
    return;
  }
  int q;
  const double r = reduce_half_pi(x, q);
  const double sk = sin_kernel(r), ck = cos_kernel(r);
  const double a = (q & 1) ? ck : sk, b = (q & 1) ? sk : ck;
  sn = (q & 2) ? -a : a;
  cs = ((q + 1) & 2) ? -b : b;
}

__device__ __forceinline__ double own_log(double x) {
  int e;
  double m = __builtin_frexp(x, &e);
  if (m < kSqrtHalf) {
    m = m * 2.0;
    e = e - 1;
  }
  const double f = (m - 1.0) / (m + 1.0);
  const double f2 = f * f;
  double p = 1.0 / 23.0;
#pragma unroll
  for (int k = 21; k >= 3; k -= 2) p = fma(p, f2, 1.0 / static_cast<double>(k));
  const double twof = 2.0 * f;
  const double lm = fma(twof, f2 * p, twof);
  const double ed = static_cast<double>(e);
  return fma(ed, kLn2Lo, lm) + ed * kLn2Hi;
}

__device__ __forceinline__ double own_exp(double x) {
  if (x < -700.0) return 0.0;
  const double k = __builtin_rint(x * kInvLn2);
  const double r = (x - k * kLn2Hi) - k * kLn2Lo;
  double p = inv_fact(14);
#pragma unroll
  for (int n = 13; n >= 1; --n) p = fma(p, r, inv_fact(n));
  return __builtin_ldexp(fma(r, p, 1.0), static_cast<int>(k));
}

// ---------------------------------------------------------------- Philox
struct U4 {
  uint32_t v[4];
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = M0 * c.v[0], hi0 = __umulhi(M0, c.v[0]);
    const uint32_t lo1 = M1 * c.v[2], hi1 = __umulhi(M1, c.v[2]);
    U4 n;
    n.v[0] = hi1 ^ c.v[1] ^ k0;
    n.v[1] = lo1;
    n.v[2] = hi0 ^ c.v[3] ^ k1;
    n.v[3] = lo0;
    c = n;
    k0 += W0;  // the bump after the last round is never used
    k1 += W1;
  }
  return c;
}

__device__ __forceinline__ double gauss(uint32_t id, uint32_t step, uint32_t tag, uint32_t key_lo,
                                        uint32_t key_hi) {
  U4 c;
  c.v[0] = id;
  c.v[1] = step;
  c.v[2] = tag;
  c.v[3] = 0u;
  const U4 w = philox4x32_10(c, key_lo, key_hi);
  const uint64_t m1 = (static_cast<uint64_t>(w.v[0] >> 5) << 26) | static_cast<uint64_t>(w.v[1] >> 6);
  const uint64_t m2 = (static_cast<uint64_t>(w.v[2] >> 5) << 26) | static_cast<uint64_t>(w.v[3] >> 6);
  const double u1 = static_cast<double>(m1 + 1u) * 0x1p-53;
  const double u2 = static_cast<double>(m2) * 0x1p-53;
  return sqrt(-2.0 * own_log(u1)) * own_cos(kTwoPi * u2);
}

}  // namespace dm
}  // namespace trk
