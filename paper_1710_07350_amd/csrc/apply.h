// apply.h -- one element applied to one particle, shared by the fused run
// kernel and the batched persistent kernel.
#pragma once
#include "elements.h"

namespace trk {

// Rarely executed handlers stay out of line so that their registers do not
// count against the hot element loop.  They take and return values, never
// references: an escaping address would place the caller's coordinate array
// in scratch memory for the whole kernel.
struct Z6 {
  double v[6];
};
static __device__ __noinline__ double radkick_call(double dp, double sigma, uint32_t pid,
                                                  uint32_t gp, uint32_t klo, uint32_t khi) {
  return fma(sigma, dm::gauss(pid, gp, 2u, klo, khi), dp);
}
static __device__ __noinline__ Z6 map_gen_call(Z6 z, const double *__restrict__ c) {
  el::map_gen(z.v, c);
  return z;
}
static __device__ __noinline__ Z6 map3_gen_call(Z6 z, const double *__restrict__ c) {
  el::map3_gen(z.v, c);
  return z;
}
__device__ __forceinline__ void call_gen(double (&z)[6], const double *c, bool third) {
  Z6 a;
#pragma unroll
  for (int k = 0; k < 6; ++k) a.v[k] = z[k];
  a = third ? map3_gen_call(a, c) : map_gen_call(a, c);
#pragma unroll
  for (int k = 0; k < 6; ++k) z[k] = a.v[k];
}

// Lattice records and constants are read-only and read at wave-uniform
// addresses: through the constant address space they are fetched with scalar
// loads into SGPRs.
#if defined(__HIP_DEVICE_COMPILE__)
#define TRK_CONST __attribute__((address_space(4)))
#else
#define TRK_CONST
#endif
typedef const DevElem TRK_CONST *ConstElems;
typedef const double TRK_CONST *ConstPool;
__device__ __forceinline__ const double *cx_pool_generic(ConstPool pool, int off) {
  return (const double *)(pool + off);
}

// What an element needs besides its record: pass-varying constants, the
// wake table and the random-number key.
struct ElemCtx {
  const double (*vc)[2];
  int nv, v0;
  const double *wake_v;
  const double *wake_par;
  uint32_t seed_lo, seed_hi;
};

// One element applied to one particle (wave-uniform record E).
template <uint32_t kFeat>
__device__ __forceinline__ void apply(const DevElem &E, ConstPool pool, const ElemCtx &cx, int p,
                                      uint32_t gp, int e, double (&z)[6], bool &alive,
                                      int64_t &rec, uint32_t pid) {
  if (!alive) return;
  ConstPool c = pool + E.off;
  switch (E.kind) {
    case K_EDRIFT: el::edrift(z, E.p0); break;
    case K_MAP2_P1: el::map_p1(z, c); break;
    case K_MAP2_P2: el::map_p2(z, c); break;
    case K_MULT: el::mult(z, E.p0, E.ip); break;
    case K_MAP2_GEN:
      if constexpr ((kFeat & F_GEN) != 0) call_gen(z, cx_pool_generic(pool, E.off), false);
      break;
    case K_MAP3_P3: el::map_p3(z, c); break;
    case K_MAP3_GEN:
      if constexpr ((kFeat & F_GEN) != 0) call_gen(z, cx_pool_generic(pool, E.off), true);
      break;
    case K_KQUAD:
      if constexpr ((kFeat & F_KD) != 0) el::kquad(z, c, E.ip);
      break;
    case K_CSBEND:
      if constexpr ((kFeat & F_KD) != 0) el::csbend(z, c, E.ip);
      break;
    case K_RFCA:
      if constexpr ((kFeat & F_RF) != 0) {
        const int v = p * cx.nv + (E.vslot - cx.v0);
        el::rfca(z, E.p0, E.p1, E.p2, E.p3, cx.vc[v][0], cx.vc[v][1]);
      }
      break;
    case K_WAKE:
      if constexpr ((kFeat & F_WAKE) != 0) {
        const int v = p * cx.nv + (E.vslot - cx.v0);
        const double vs = el::wake_interp(z[4], cx.wake_par[0], cx.wake_par[1], cx.wake_v, E.ip);
        z[5] = fma(-cx.vc[v][0], vs, z[5]);
      }
      break;
    case K_TRWAKE:
      if constexpr ((kFeat & F_WAKE) != 0) {
        const int v = p * cx.nv + (E.vslot - cx.v0);
        const double ux = el::wake_interp(z[4], cx.wake_par[0], cx.wake_par[1], cx.wake_v, E.ip);
        const double uy =
            el::wake_interp(z[4], cx.wake_par[0], cx.wake_par[1], cx.wake_v + E.ip, E.ip);
        el::trwake(z, cx.vc[v][0], ux, uy);
      }
      break;
    case K_RADKICK:
      if constexpr ((kFeat & F_RNG) != 0)
        z[5] = radkick_call(z[5], E.p0, pid, gp, cx.seed_lo, cx.seed_hi);
      break;
    default: break;
  }
  if (E.aper != TRK_APER_NONE && el::aperture_lost(E.aper, E.a0, E.a1, z)) {
    alive = false;
    rec = static_cast<int64_t>((static_cast<uint64_t>(gp) << 32) | static_cast<uint32_t>(e));
  }
}

// Runs that touch only s and delta (RF cavities, wake kicks, maps whose other
// rows are identities, markers; no apertures): the arithmetic of apply() on
// the two coordinates, without the registers of the other element kinds,
// applied to kP particles at once (lanes with on[q] false keep their values).
template <uint32_t kFeat, int kP>
__device__ __forceinline__ void apply_long_q(const DevElem &E, ConstPool pool, const ElemCtx &cx,
                                             int p, double (&s)[kP], double (&d)[kP],
                                             const bool (&on)[kP]) {
  switch (E.kind) {
    case K_MAP2_P2: {
      ConstPool c = pool + E.off;
      const double r55 = c[4], r56 = c[5], r66 = c[6], t566 = c[7];
#pragma unroll
      for (int q = 0; q < kP; ++q) {
        double a = r55 * s[q];
        a = fma(r56, d[q], a);
        a = fma(t566, d[q] * d[q], a);
        if (on[q]) {
          s[q] = a;
          d[q] = r66 * d[q];
        }
      }
      break;
    }
    case K_RFCA:
      if constexpr ((kFeat & F_RF) != 0) {
        const int v = p * cx.nv + (E.vslot - cx.v0);
        const double pin = cx.vc[v][0], inv_pout = cx.vc[v][1];
#pragma unroll
        for (int q = 0; q < kP; ++q)
          if (on[q]) {
            double z[6] = {0.0, 0.0, 0.0, 0.0, s[q], d[q]};
            el::rfca(z, E.p0, E.p1, E.p2, E.p3, pin, inv_pout);
            d[q] = z[5];
          }
      }
      break;
    case K_WAKE:
      if constexpr ((kFeat & F_WAKE) != 0) {
        const int v = p * cx.nv + (E.vslot - cx.v0);
        const double kf = cx.vc[v][0];
        const double smin = cx.wake_par[0], inv = cx.wake_par[1];
        int i0[kP];
        double w[kP], v0[kP], v1[kP];
        // positions first, then every table read, then the kicks: the reads
        // of all kP particles are in flight together (indices stay in
        // [0, nbins - 2] for any s, so no lane reads out of bounds)
#pragma unroll
        for (int q = 0; q < kP; ++q) el::wake_pos(s[q], smin, inv, E.ip, i0[q], w[q]);
#pragma unroll
        for (int q = 0; q < kP; ++q) {
          v0[q] = cx.wake_v[i0[q]];
          v1[q] = cx.wake_v[i0[q] + 1];
        }
#pragma unroll
        for (int q = 0; q < kP; ++q) {
          const double vs = fma(w[q], v1[q] - v0[q], v0[q]);
          if (on[q]) d[q] = fma(-kf, vs, d[q]);
        }
      }
      break;
    default: break;
  }
}

}  // namespace trk
