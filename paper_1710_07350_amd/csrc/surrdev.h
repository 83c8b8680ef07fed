// surrdev.h -- per-particle arithmetic of the section surrogate shared by
// the .hip translation units: the admission gate, the linear part C + R z
// and the sampler's draw.  Every operation is a separate binary64 rounding
// (no contraction), in a fixed order, so that the gate's decision and the
// linear part are reproducible bit for bit on any IEEE machine.
#pragma once
#include "devmath.h"
#include "mlp.h"

namespace trk {

constexpr uint32_t kTagSample = 5;  // Philox counter tag of the sampler

// Linear Courant--Snyder amplitude bound.  Admitted iff inside the box
// |z_k| <= hw_k (k != s) and (xhat/a)^2 + (yhat/b)^2 <= (1 - margin)^2 with
// xhat = sqrt(J_x betahat_x) + etahat |delta|, yhat = sqrt(J_y betahat_y),
// J = gamma u^2 + 2 alpha u u' + beta u'^2 of the betatron part.
__device__ __forceinline__ bool surr_gate(const SurrDev &c, const double (&z)[6]) {
  bool box = true;
#pragma unroll
  for (int k = 0; k < 6; ++k)
    if (k != kMlpSCol) box = box && fabs(z[k]) <= c.hw[k];
  const double xb = z[0] - c.eta * z[5];
  const double xpb = z[1] - c.etap * z[5];
  const double jx = ((c.gx * xb) * xb + (c.ax2 * xb) * xpb) + (c.bx * xpb) * xpb;
  const double jy = ((c.gy * z[2]) * z[2] + (c.ay2 * z[2]) * z[3]) + (c.by * z[3]) * z[3];
  const double xh = sqrt(fmax(jx * c.bhx, 0.0)) + c.eh * fabs(z[5]);
  const double yh = sqrt(fmax(jy * c.bhy, 0.0));
  const double ux = xh * c.inv_a;
  const double uy = yh * c.inv_b;
  const double q = ux * ux + uy * uy;
  return box && q <= c.lim;
}

// C + R z per output: ((C_i + R_i0 z_0) + R_i1 z_1) + ..., zero terms skipped
__device__ __forceinline__ double surr_linear(const SurrDev &c, const double (&z)[6], int i) {
  double acc = c.C[i];
#pragma unroll
  for (int j = 0; j < 6; ++j)
    if (c.R[6 * i + j] != 0.0) acc = acc + c.R[6 * i + j] * z[j];
  return acc;
}

// candidate `cand` of the sampler: two Philox4x32-10 blocks with counters
// (cand_lo, cand_hi, kTagSample, 0|1), key = seed; z_k = (2 u_k - 1) sw_k with
// u_k = (w_k + 1/2) 2^-32.
__device__ __forceinline__ void surr_draw(const SurrDev &c, uint64_t seed, uint64_t cand,
                                          double (&z)[6]) {
  dm::U4 a, b;
  a.v[0] = b.v[0] = static_cast<uint32_t>(cand);
  a.v[1] = b.v[1] = static_cast<uint32_t>(cand >> 32);
  a.v[2] = b.v[2] = kTagSample;
  a.v[3] = 0u;
  b.v[3] = 1u;
  const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
  const dm::U4 wa = dm::philox4x32_10(a, k0, k1);
  const dm::U4 wb = dm::philox4x32_10(b, k0, k1);
  const uint32_t w[6] = {wa.v[0], wa.v[1], wa.v[2], wa.v[3], wb.v[0], wb.v[1]};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double u = (static_cast<double>(w[k]) + 0.5) * 0x1p-32;
    z[k] = (2.0 * u - 1.0) * c.sw[k];
  }
}

}  // namespace trk
