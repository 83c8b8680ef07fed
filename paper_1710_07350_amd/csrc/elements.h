// elements.h -- per-particle element maps (device).
//
// z = (x, x', y, y', s, delta).  Each map fixes its operation order; fma
// appears only where written (the library is built without contraction).
// Physical content, by element (the element table of Sec. 3 of the paper):
//   EDRIFT  exact drift (Sec. 2.1 listings): x += x'L, y += y'L and the path
//           excess L(sqrt(1+u) - 1) = L u / (1 + sqrt(1+u)), u = x'^2 + y'^2.
//   MAP2    z_i = C_i + sum_j R_ij z_j + sum_{j<=k} T_ijk z_j z_k from the
//           input vector: non-zero terms only, order C, R by ascending j, T by
//           ascending (j,k); the first term starts the sum (coefficient times
//           coordinates), each later term is added with one fma; products
//           z_j z_k rounded once.  A row whose only term is R_ii = 1 is exact.
//   MAP3    MAP2, then sum_{j<=k<=l} U_ijkl z_j z_k z_l, (j,k,l) ascending,
//           each monomial rounded as (z_j z_k) z_l (the M3 matrix tracking).
//   MULT    thin kick Delta px - i Delta py = -(KnL/n!)(x+iy)^n on canonical
//           px = x'(1+delta)/sqrt(1+x'^2+y'^2), back to x' = px/pz.
//   KQUAD   4th-order symplectic kick-drift (Yoshida): kicks
//           Delta px = -l k1 x, Delta py = +l k1 y, canonical exact drifts.
//   CSBEND  the sector-bend Hamiltonian -(1+hx)pz + hx + h^2x^2/2 split into
//           a curved-frame drift (straight line, solved in polar form) and the
//           kick Delta px = -l h (1 + hx).
//   RFCA    zero-length cavity: delta <- (delta P + V (cos(phi+ks) - cos phi))/P',
//           P' = P + V cos phi, the difference as -2 sin(phi+ks/2) sin(ks/2).
//   TRWAKE  canonical px, py gain kfac V_x(s), kfac V_y(s) (as in MULT).
#pragma once
#include "devmath.h"
#include "trk_internal.h"

namespace trk {
namespace el {

__device__ __forceinline__ void edrift(double (&z)[6], double L) {
  const double xp = z[1], yp = z[3];
  const double u = fma(xp, xp, yp * yp);
  z[0] = fma(xp, L, z[0]);
  z[2] = fma(yp, L, z[2]);
  z[4] = fma(L, u / (1.0 + sqrt(1.0 + u)), z[4]);
}

// thick-quad sparsity pattern: every listed coefficient is non-zero
template <class CP>
__device__ __forceinline__ void map_p1(double (&z)[6], CP c) {
  const double x = z[0], xp = z[1], y = z[2], yp = z[3], s = z[4], d = z[5];
  const double xd = x * d, xpd = xp * d, yd = y * d, ypd = yp * d;
  double a;
  a = c[0] * x; a = fma(c[1], xp, a); a = fma(c[2], xd, a); a = fma(c[3], xpd, a);
  z[0] = a;
  a = c[4] * x; a = fma(c[5], xp, a); a = fma(c[6], xd, a); a = fma(c[7], xpd, a);
  z[1] = a;
  a = c[8] * y; a = fma(c[9], yp, a); a = fma(c[10], yd, a); a = fma(c[11], ypd, a);
  z[2] = a;
  a = c[12] * y; a = fma(c[13], yp, a); a = fma(c[14], yd, a); a = fma(c[15], ypd, a);
  z[3] = a;
  a = c[16] * s;
  a = fma(c[17], x * x, a);
  a = fma(c[18], x * xp, a);
  a = fma(c[19], xp * xp, a);
  a = fma(c[20], y * y, a);
  a = fma(c[21], y * yp, a);
  a = fma(c[22], yp * yp, a);
  z[4] = a;
  z[5] = c[23] * d;
}

// identity + R56 + T566 (a chicane)
template <class CP>
__device__ __forceinline__ void map_p2(double (&z)[6], CP c) {
  const double s = z[4], d = z[5];
  z[0] = c[0] * z[0];
  z[1] = c[1] * z[1];
  z[2] = c[2] * z[2];
  z[3] = c[3] * z[3];
  double a = c[4] * s;
  a = fma(c[5], d, a);
  a = fma(c[7], d * d, a);
  z[4] = a;
  z[5] = c[6] * d;
}

// the third-order thick-quad pattern: P1's terms, then the chromatic cubic
// ones, each monomial rounded as (z_j z_k) z_l
template <class CP>
__device__ __forceinline__ void map_p3(double (&z)[6], CP c) {
  const double x = z[0], xp = z[1], y = z[2], yp = z[3], s = z[4], d = z[5];
  const double xd = x * d, xpd = xp * d, yd = y * d, ypd = yp * d;
  double a;
  a = c[0] * x; a = fma(c[1], xp, a); a = fma(c[2], xd, a); a = fma(c[3], xpd, a);
  a = fma(c[24], xd * d, a); a = fma(c[25], xpd * d, a);
  z[0] = a;
  a = c[4] * x; a = fma(c[5], xp, a); a = fma(c[6], xd, a); a = fma(c[7], xpd, a);
  a = fma(c[26], xd * d, a); a = fma(c[27], xpd * d, a);
  z[1] = a;
  a = c[8] * y; a = fma(c[9], yp, a); a = fma(c[10], yd, a); a = fma(c[11], ypd, a);
  a = fma(c[28], yd * d, a); a = fma(c[29], ypd * d, a);
  z[2] = a;
  a = c[12] * y; a = fma(c[13], yp, a); a = fma(c[14], yd, a); a = fma(c[15], ypd, a);
  a = fma(c[30], yd * d, a); a = fma(c[31], ypd * d, a);
  z[3] = a;
  const double xx = x * x, xxp = x * xp, xpxp = xp * xp;
  const double yy = y * y, yyp = y * yp, ypyp = yp * yp;
  a = c[16] * s;
  a = fma(c[17], xx, a);
  a = fma(c[18], xxp, a);
  a = fma(c[19], xpxp, a);
  a = fma(c[20], yy, a);
  a = fma(c[21], yyp, a);
  a = fma(c[22], ypyp, a);
  a = fma(c[32], xx * d, a);
  a = fma(c[33], xxp * d, a);
  a = fma(c[34], xpxp * d, a);
  a = fma(c[35], yy * d, a);
  a = fma(c[36], yyp * d, a);
  a = fma(c[37], ypyp * d, a);
  z[4] = a;
  z[5] = c[23] * d;
}

// any third-order map: as map_gen, then the cubic terms (j,k,l) ascending.
// Loops run over monomials (rolled, with wave-uniform indices from a table)
// with the six rows inside, so a monomial is formed once and consumed at
// once and the evaluator keeps few registers; every row still adds its terms
// in the order C, R, T, U, each group ascending.
struct Triple {
  unsigned char j, k, l;
};
struct TripleTable {
  Triple t[56];
  constexpr TripleTable() : t{} {
    int q = 0;
    for (int j = 0; j < 6; ++j)
      for (int k = j; k < 6; ++k)
        for (int l = k; l < 6; ++l, ++q)
          t[q] = Triple{static_cast<unsigned char>(j), static_cast<unsigned char>(k),
                        static_cast<unsigned char>(l)};
  }
};
__device__ __forceinline__ double pick6(const double (&v)[6], int j) {
  return j == 0 ? v[0] : j == 1 ? v[1] : j == 2 ? v[2] : j == 3 ? v[3] : j == 4 ? v[4] : v[5];
}

template <class CP>
__device__ __forceinline__ void map3_gen(double (&z)[6], CP c) {
  constexpr TripleTable kTri;
  double in[6], a[6];
  bool have[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    in[i] = z[i];
    const double ci = c[i];
    have[i] = ci != 0.0;
    a[i] = have[i] ? ci : 0.0;
  }
  auto add = [&](int i, double coef, double m) {
    if (coef != 0.0) {
      a[i] = have[i] ? fma(coef, m, a[i]) : coef * m;
      have[i] = true;
    }
  };
#pragma unroll
  for (int j = 0; j < 6; ++j)
#pragma unroll
    for (int i = 0; i < 6; ++i) add(i, c[6 + 6 * i + j], in[j]);
  int p = 0;
#pragma unroll
  for (int j = 0; j < 6; ++j)
#pragma unroll
    for (int k = j; k < 6; ++k, ++p) {
      const double m = in[j] * in[k];
#pragma unroll
      for (int i = 0; i < 6; ++i) add(i, c[42 + 21 * i + p], m);
    }
#pragma unroll 1
  for (int q = 0; q < 56; ++q) {
    const Triple tr = kTri.t[q];
    const double m = (pick6(in, tr.j) * pick6(in, tr.k)) * pick6(in, tr.l);
#pragma unroll
    for (int i = 0; i < 6; ++i) add(i, c[168 + 56 * i + q], m);
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) z[i] = a[i];
}

// any second-order map: coefficient tests are wave-uniform branches
template <class CP>
__device__ __forceinline__ void map_gen(double (&z)[6], CP c) {
  double in[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) in[k] = z[k];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double a = 0.0;
    bool have = false;
    const double ci = c[i];
    if (ci != 0.0) {
      a = ci;
      have = true;
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const double r = c[6 + 6 * i + j];
      if (r != 0.0) {
        a = have ? fma(r, in[j], a) : r * in[j];
        have = true;
      }
    }
    int p = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j)
#pragma unroll
      for (int k = j; k < 6; ++k, ++p) {
        const double t = c[42 + 21 * i + p];
        if (t != 0.0) {
          const double m = in[j] * in[k];
          a = have ? fma(t, m, a) : t * m;
          have = true;
        }
      }
    z[i] = a;
  }
}

struct Canon {
  double px, py, opd, opd2;
};

__device__ __forceinline__ Canon canonical(const double (&z)[6]) {
  Canon c;
  c.opd = 1.0 + z[5];
  c.opd2 = c.opd * c.opd;
  const double xp = z[1], yp = z[3];
  const double u = fma(xp, xp, yp * yp);
  const double pz = c.opd / sqrt(1.0 + u);
  c.px = xp * pz;
  c.py = yp * pz;
  return c;
}

__device__ __forceinline__ void slopes(double (&z)[6], const Canon &c) {
  const double q = fma(c.px, c.px, c.py * c.py);
  const double pz = sqrt(c.opd2 - q);
  const double r = 1.0 / pz;
  z[1] = c.px * r;
  z[3] = c.py * r;
}

__device__ __forceinline__ void mult(double (&z)[6], double kn, int order) {
  Canon c = canonical(z);
  const double x = z[0], y = z[2];
  double re = x, im = y;
  for (int m = 2; m <= order; ++m) {
    const double nre = (re * x) - (im * y);
    const double nim = (re * y) + (im * x);
    re = nre;
    im = nim;
  }
  c.px = fma(-kn, re, c.px);
  c.py = fma(kn, im, c.py);
  slopes(z, c);
}

// TRWAKE: the canonical momenta gain kfac V_x and kfac V_y
__device__ __forceinline__ void trwake(double (&z)[6], double kfac, double ux, double uy) {
  Canon c = canonical(z);
  c.px = fma(kfac, ux, c.px);
  c.py = fma(kfac, uy, c.py);
  slopes(z, c);
}

// x, y advance by dl px/pz, dl py/pz and s by the cancellation-free excess
// dl q / (pz (opd + pz)): both from the one quotient w = dl / (pz (opd + pz))
__device__ __forceinline__ void canon_drift(double (&z)[6], Canon &c, double dl) {
  const double q = fma(c.px, c.px, c.py * c.py);
  const double pz = sqrt(c.opd2 - q);
  const double a = c.opd + pz;
  const double w = dl / (pz * a);
  const double t = a * w;
  z[0] = fma(c.px, t, z[0]);
  z[2] = fma(c.py, t, z[2]);
  z[4] = fma(q, w, z[4]);
}

template <class CP>
__device__ __forceinline__ void kquad(double (&z)[6], CP k, int nsteps) {
  Canon c = canonical(z);
  for (int st = 0; st < nsteps; ++st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const double kq = k[i];
      c.px = fma(-kq, z[0], c.px);
      c.py = fma(kq, z[2], c.py);
      if (i < 3) canon_drift(z, c, k[4 + i]);
    }
  }
  slopes(z, c);
}

template <class CP>
__device__ __forceinline__ void csbend(double (&z)[6], CP k, int nsteps) {
  Canon c = canonical(z);
  const double iopd = 1.0 / c.opd;
  for (int st = 0; st < nsteps; ++st) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      c.px = c.px - fma(k[4 + i], z[0], k[i]);
      if (i < 3) {
        const double cph = k[8 + i], sph = k[11 + i], vers = k[14 + i], rs = k[17 + i];
        const double arc = k[20 + i];
        const double x = z[0];
        const double q = fma(c.px, c.px, c.py * c.py);
        const double pz = sqrt(c.opd2 - q);
        const double pxn = fma(c.px, cph, pz * sph);
        const double pzn = fma(pz, cph, -(c.px * sph));
        const double tau = (fma(x, sph, rs) * c.opd) / pzn;
        const double g = tau * iopd;
        z[0] = fma(g, pxn, fma(x, cph, -vers));
        z[2] = fma(g, c.py, z[2]);
        z[4] = z[4] + (tau - arc);
        c.px = pxn;
      }
    }
  }
  slopes(z, c);
}

// a = ks/2: cos(phase + ks) - cos(phase) = -2 sin(a) (sin(phase) cos(a) + cos(phase) sin(a))
__device__ __forceinline__ void rfca(double (&z)[6], double hk, double sph, double cph,
                                     double volt, double pin, double inv_pout) {
  const double a = hk * z[4];
  double sa, ca;
  dm::own_sincos(a, sa, ca);
  const double dc = (-2.0 * fma(sph, ca, cph * sa)) * sa;
  const double num = fma(z[5], pin, volt * dc);
  z[5] = num * inv_pout;
}

// V(s): linear between bin centres, constant beyond the first and last.
// wake_pos gives the left bin i0 (always in [0, nbins - 2]) and the weight w.
__device__ __forceinline__ void wake_pos(double s, double smin, double inv, int nbins, int &i0,
                                         double &w) {
  const double f = (s - smin) * inv - 0.5;
  const double fl = floor(f);
  if (!(fl >= 0.0))
    i0 = 0;
  else if (fl > static_cast<double>(nbins - 2))
    i0 = nbins - 2;
  else
    i0 = static_cast<int>(fl);
  w = f - static_cast<double>(i0);
  if (!(w >= 0.0)) w = 0.0;
  if (w > 1.0) w = 1.0;
}

__device__ __forceinline__ double wake_interp(double s, double smin, double inv,
                                              const double *__restrict__ v, int nbins) {
  int i0;
  double w;
  wake_pos(s, smin, inv, nbins, i0, w);
  const double v0 = v[i0];
  return fma(w, v[i0 + 1] - v0, v0);
}

__device__ __forceinline__ bool aperture_lost(int aper, double a0, double a1, const double (&z)[6]) {
  if (aper == TRK_APER_RECT) return !(fabs(z[0]) < a0 && fabs(z[2]) < a1);
  const double xa = z[0] * a0, ya = z[2] * a1;
  const double q = fma(xa, xa, ya * ya);
  return !(q < 1.0);
}

}  // namespace el
}  // namespace trk
