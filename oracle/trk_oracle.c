/* trk_oracle.c -- plain, slow, CPU oracle of lumped-element tracking.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.
 *
 * Structure follows the paper's description of tracking (Sec. 2 and the
 * element table of Sec. 3): the beam passes element by element; each element
 * is a per-particle update, except the collective wake element, which first
 * builds a histogram of s (Sec. 2.2), convolves it with the wake function
 * (Sec. 2.3) and then kicks every particle.  Losses are recorded per particle
 * (Sec. 2.5) and the arrays are reordered once at the end.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (no contraction: every fma
 * below is explicit).  The particle loops are independent, so the optional
 * OpenMP parallelisation does not change any result; every reduction runs
 * serially.
 */
#include "trk_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define C_LIGHT 299792458.0
#define TWO_PI 0x1.921fb54442d18p+2

/* ======================================================================
 * Own elementary functions.
 * sin/cos: Cody & Waite (1980) three-part reduction by pi/2 (the first two
 * parts carry 33 significant bits so k*part is exact for |k| < 2^20), then
 * Taylor polynomials on |r| <= pi/4 with coefficients (-1)^k / n!, each the
 * correctly rounded quotient 1/n! (n! is exact in binary64 for n <= 22).
 * log: x = 2^e m, m in [sqrt(1/2), sqrt(2)); log m = 2 atanh((m-1)/(m+1))
 * as an odd series with coefficients 1/(2k+1); e*ln2 from a two-part ln2.
 * exp: x = k ln2 + r, |r| <= ln2/2, Taylor to degree 14, scaled by 2^k.
 * ====================================================================== */
static const double PIO2_HI = 0x1.921fb54400000p+0;
static const double PIO2_MID = 0x1.0b4611a600000p-34;
static const double PIO2_LO = 0x1.3198a2e037073p-69;
static const double TWO_OVER_PI = 0x1.45f306dc9c883p-1;
static const double LN2_HI = 0x1.62e42ff000000p-1;
static const double LN2_LO = -0x1.718432a1b0e26p-35;
static const double INV_LN2 = 0x1.71547652b82fep+0;
static const double SQRT_HALF = 0x1.6a09e667f3bcdp-1;

static double fact(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= (double)i; /* exact for n <= 22 */
  return f;
}

/* sin(r) and cos(r) for |r| <= pi/4 */
static double sin_poly(double r) {
  double r2 = r * r;
  double p = 1.0 / fact(17);
  p = fma(p, r2, -1.0 / fact(15));
  p = fma(p, r2, 1.0 / fact(13));
  p = fma(p, r2, -1.0 / fact(11));
  p = fma(p, r2, 1.0 / fact(9));
  p = fma(p, r2, -1.0 / fact(7));
  p = fma(p, r2, 1.0 / fact(5));
  p = fma(p, r2, -1.0 / fact(3));
  return fma(r * r2, p, r);
}
static double cos_poly(double r) {
  double r2 = r * r;
  double p = -1.0 / fact(18);
  p = fma(p, r2, 1.0 / fact(16));
  p = fma(p, r2, -1.0 / fact(14));
  p = fma(p, r2, 1.0 / fact(12));
  p = fma(p, r2, -1.0 / fact(10));
  p = fma(p, r2, 1.0 / fact(8));
  p = fma(p, r2, -1.0 / fact(6));
  p = fma(p, r2, 1.0 / fact(4));
  p = fma(p, r2, -1.0 / fact(2));
  return fma(r2, p, 1.0);
}
/* reduce x to r in [-pi/4, pi/4] and the quadrant k mod 4 */
static double reduce_pio2(double x, int *quadrant) {
  double kd = rint(x * TWO_OVER_PI);
  double r = ((x - kd * PIO2_HI) - kd * PIO2_MID) - kd * PIO2_LO;
  long long k = (long long)kd;
  *quadrant = (int)(k & 3);
  return r;
}
double orc_sin(double x) {
  int q;
  double r = reduce_pio2(x, &q);
  switch (q) {
    case 0: return sin_poly(r);
    case 1: return cos_poly(r);
    case 2: return -sin_poly(r);
    default: return -cos_poly(r);
  }
}
double orc_cos(double x) {
  int q;
  double r = reduce_pio2(x, &q);
  switch (q) {
    case 0: return cos_poly(r);
    case 1: return -sin_poly(r);
    case 2: return -cos_poly(r);
    default: return sin_poly(r);
  }
}
double orc_log(double x) {
  int e;
  double m = frexp(x, &e); /* x = m 2^e, m in [0.5, 1) */
  if (m < SQRT_HALF) {
    m = m * 2.0;
    e = e - 1;
  }
  double f = (m - 1.0) / (m + 1.0);
  double f2 = f * f;
  double p = 1.0 / 23.0;
  p = fma(p, f2, 1.0 / 21.0);
  p = fma(p, f2, 1.0 / 19.0);
  p = fma(p, f2, 1.0 / 17.0);
  p = fma(p, f2, 1.0 / 15.0);
  p = fma(p, f2, 1.0 / 13.0);
  p = fma(p, f2, 1.0 / 11.0);
  p = fma(p, f2, 1.0 / 9.0);
  p = fma(p, f2, 1.0 / 7.0);
  p = fma(p, f2, 1.0 / 5.0);
  p = fma(p, f2, 1.0 / 3.0);
  double twof = 2.0 * f;
  double lm = fma(twof, f2 * p, twof);
  double ed = (double)e;
  return fma(ed, LN2_LO, lm) + ed * LN2_HI;
}
double orc_exp(double x) {
  if (x < -700.0) return 0.0;
  double kd = rint(x * INV_LN2);
  double r = (x - kd * LN2_HI) - kd * LN2_LO;
  double p = 1.0 / fact(14);
  for (int n = 13; n >= 1; --n) p = fma(p, r, 1.0 / fact(n));
  double er = fma(r, p, 1.0);
  return ldexp(er, (int)kd);
}

/* ======================================================================
 * Philox4x32-10: Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11.  A round multiplies counter words 0 and 2 by the
 * two round multipliers (high and low 32-bit halves), xors the high halves
 * with the other two words and the key; the key advances by the two Weyl
 * increments between rounds.
 * ====================================================================== */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* One standard normal per counter (id, step, tag, 0) and key (seed lo, hi):
 * two 53-bit uniforms u1 in (0,1], u2 in [0,1), g = sqrt(-2 ln u1) cos(2 pi u2). */
double orc_gauss(uint32_t id, uint32_t step, uint32_t tag, uint64_t seed) {
  uint32_t ctr[4] = {id, step, tag, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  uint64_t m1 = ((uint64_t)(w[0] >> 5) << 26) | (uint64_t)(w[1] >> 6);
  uint64_t m2 = ((uint64_t)(w[2] >> 5) << 26) | (uint64_t)(w[3] >> 6);
  double u1 = (double)(m1 + 1u) * 0x1p-53;
  double u2 = (double)m2 * 0x1p-53;
  return sqrt(-2.0 * orc_log(u1)) * orc_cos(TWO_PI * u2);
}

/* ======================================================================
 * Element constants
 * ====================================================================== */

/* Fourth-order symplectic integrator (Yoshida 1990; Forest & Ruth 1990) in
 * kick-drift-kick form: kicks c = (w1/2, (w0+w1)/2, (w0+w1)/2, w1/2),
 * drifts d = (w1, w0, w1), w1 = 1/(2 - 2^(1/3)), w0 = -2^(1/3)/(2 - 2^(1/3)). */
void orc_yoshida(double c[4], double d[3]) {
  /* 2^(1/3) correctly rounded (not libm's cbrt, which may differ by an ulp
   * between a compile-time fold and a run-time call) */
  double cr = 0x1.428a2f98d728bp+0;
  double w1 = 1.0 / (2.0 - cr);
  double w0 = -cr / (2.0 - cr);
  c[0] = 0.5 * w1;
  c[1] = 0.5 * (w0 + w1);
  c[2] = 0.5 * (w0 + w1);
  c[3] = 0.5 * w1;
  d[0] = w1;
  d[1] = w0;
  d[2] = w1;
}

/* index of the pair (j,k), j<=k, in the 21 second-order monomials */
static int pair_index(int j, int k) {
  int idx = 0;
  for (int a = 0; a < 6; ++a)
    for (int b = a; b < 6; ++b) {
      if (a == j && b == k) return idx;
      ++idx;
    }
  return -1;
}

/* Thick quadrupole as a second-order transfer map (the paper's matrix
 * tracking of QUAD, element table): paraxial motion x'' = -K x, y'' = +K y
 * with K = k1/(1+delta).  First order is the usual cos/sin (cosh/sinh)
 * matrix; the T_ij6 terms are its first derivative in delta; the T_5jk path
 * terms integrate (x'^2 + y'^2)/2 along the linear orbit. */
void orc_quad_coef(double L, double k1, double coef[168]) {
  memset(coef, 0, 168 * sizeof(double));
  double *R = coef + 6;   /* R[i*6+j] */
  double *T = coef + 42;  /* T[i*21+pair] */
  R[4 * 6 + 4] = 1.0;
  R[5 * 6 + 5] = 1.0;
  if (k1 == 0.0) {
    R[0 * 6 + 0] = 1.0; R[0 * 6 + 1] = L; R[1 * 6 + 1] = 1.0;
    R[2 * 6 + 2] = 1.0; R[2 * 6 + 3] = L; R[3 * 6 + 3] = 1.0;
    T[4 * 21 + pair_index(1, 1)] = 0.5 * L;
    T[4 * 21 + pair_index(3, 3)] = 0.5 * L;
    return;
  }
  double w = sqrt(fabs(k1));
  double phi = w * L;
  double cf = cos(phi), sf = sin(phi), s2f = sin(2.0 * phi);
  double ch = cosh(phi), sh = sinh(phi), sh2 = sinh(2.0 * phi);
  /* focusing plane: [R11 R12 R21 R22], [T16 T26 T'16 T'26], [T511 T512 T522] */
  double fR[4] = {cf, sf / w, -w * sf, cf};
  double fT[4] = {(0.5 * phi) * sf, (sf - phi * cf) / (2.0 * w),
                  (0.5 * w) * (sf + phi * cf), (0.5 * phi) * sf};
  double fS[3] = {(0.5 * (w * w)) * (0.5 * L - s2f / (4.0 * w)), -0.5 * (sf * sf),
                  0.5 * (0.5 * L + s2f / (4.0 * w))};
  double dR[4] = {ch, sh / w, w * sh, ch};
  double dT[4] = {-((0.5 * phi) * sh), (sh - phi * ch) / (2.0 * w),
                  -((0.5 * w) * (sh + phi * ch)), -((0.5 * phi) * sh)};
  double dS[3] = {(0.5 * (w * w)) * (sh2 / (4.0 * w) - 0.5 * L), 0.5 * (sh * sh),
                  0.5 * (0.5 * L + sh2 / (4.0 * w))};
  const double *xR = k1 > 0 ? fR : dR, *xT = k1 > 0 ? fT : dT, *xS = k1 > 0 ? fS : dS;
  const double *yR = k1 > 0 ? dR : fR, *yT = k1 > 0 ? dT : fT, *yS = k1 > 0 ? dS : fS;
  for (int p = 0; p < 2; ++p) {
    int o = 2 * p; /* plane offset: 0 for x, 2 for y */
    const double *pr = p == 0 ? xR : yR, *pt = p == 0 ? xT : yT, *ps = p == 0 ? xS : yS;
    R[(o + 0) * 6 + o + 0] = pr[0];
    R[(o + 0) * 6 + o + 1] = pr[1];
    R[(o + 1) * 6 + o + 0] = pr[2];
    R[(o + 1) * 6 + o + 1] = pr[3];
    T[(o + 0) * 21 + pair_index(o + 0, 5)] = pt[0];
    T[(o + 0) * 21 + pair_index(o + 1, 5)] = pt[1];
    T[(o + 1) * 21 + pair_index(o + 0, 5)] = pt[2];
    T[(o + 1) * 21 + pair_index(o + 1, 5)] = pt[3];
    T[4 * 21 + pair_index(o + 0, o + 0)] = ps[0];
    T[4 * 21 + pair_index(o + 0, o + 1)] = ps[1];
    T[4 * 21 + pair_index(o + 1, o + 1)] = ps[2];
  }
}

/* index of the monomial z_j z_k z_l, j <= k <= l, among the 56 cubic ones
 * in lexicographic order (0,0,0), (0,0,1), ..., (5,5,5) */
static int triple_index(int j, int k, int l) {
  int n = 0;
  for (int a = 0; a < 6; ++a)
    for (int b = a; b < 6; ++b)
      for (int c = b; c < 6; ++c) {
        if (a == j && b == k && c == l) return n;
        ++n;
      }
  return -1;
}

/* Thick quadrupole to third order in the same paraxial model (x'' = -K x,
 * y'' = K y, K = k1/(1+delta), s' = (x'^2 + y'^2)/2): the first 168
 * coefficients as orc_quad_coef, then U[6][56].  The model is linear in
 * the transverse coordinates, so the cubic terms are chromatic:
 *   U_{i,j,6,6} = (1/2) d^2 R_ij / d delta^2   (i, j in one plane),
 *   U_{5,j,k,6} = d T_5jk / d delta,
 * with phi = omega L and omega = sqrt(|k1|/(1+delta)), so that
 * d phi/d delta = -phi/2 and d^2 phi/d delta^2 = 3 phi/4 at delta = 0. */
void orc_quad3_coef(double L, double k1, double coef[504]) {
  memset(coef, 0, 504 * sizeof(double));
  orc_quad_coef(L, k1, coef);
  if (k1 == 0.0) return;
  double *U = coef + 168; /* U[i*56 + triple] */
  double w = sqrt(fabs(k1));
  double f = w * L;
  double cf = cos(f), sf = sin(f), c2 = cos(2.0 * f), s2 = sin(2.0 * f);
  double ch = cosh(f), sh = sinh(f), ch2 = cosh(2.0 * f), sh2 = sinh(2.0 * f);
  double f2 = f * f;
  /* focusing plane: U for [R11 R12 R21 R22] and [T511 T512 T522] */
  double fU[4] = {-(f2 / 8.0) * cf - (3.0 * f / 8.0) * sf,
                  ((f * cf - sf) - f2 * sf) / (8.0 * w),
                  -(w / 8.0) * ((5.0 * f * cf + 3.0 * sf) - f2 * sf),
                  -(f2 / 8.0) * cf - (3.0 * f / 8.0) * sf};
  double fS[3] = {-(w / 16.0) * ((4.0 * f - s2) - 2.0 * f * c2), (f * s2) / 4.0,
                  -(2.0 * f * c2 - s2) / (16.0 * w)};
  /* defocusing plane */
  double dU[4] = {(f2 / 8.0) * ch + (3.0 * f / 8.0) * sh,
                  ((f2 * sh + f * ch) - sh) / (8.0 * w),
                  (w / 8.0) * ((5.0 * f * ch + 3.0 * sh) + f2 * sh),
                  (f2 / 8.0) * ch + (3.0 * f / 8.0) * sh};
  double dS[3] = {-(w / 16.0) * ((sh2 + 2.0 * f * ch2) - 4.0 * f), -(f * sh2) / 4.0,
                  -(2.0 * f * ch2 - sh2) / (16.0 * w)};
  const double *xU = k1 > 0 ? fU : dU, *xS = k1 > 0 ? fS : dS;
  const double *yU = k1 > 0 ? dU : fU, *yS = k1 > 0 ? dS : fS;
  for (int p = 0; p < 2; ++p) {
    int o = 2 * p;
    const double *pu = p == 0 ? xU : yU, *ps = p == 0 ? xS : yS;
    U[(o + 0) * 56 + triple_index(o + 0, 5, 5)] = pu[0];
    U[(o + 0) * 56 + triple_index(o + 1, 5, 5)] = pu[1];
    U[(o + 1) * 56 + triple_index(o + 0, 5, 5)] = pu[2];
    U[(o + 1) * 56 + triple_index(o + 1, 5, 5)] = pu[3];
    U[4 * 56 + triple_index(o + 0, o + 0, 5)] = ps[0];
    U[4 * 56 + triple_index(o + 0, o + 1, 5)] = ps[1];
    U[4 * 56 + triple_index(o + 1, o + 1, 5)] = ps[2];
  }
}

/* ======================================================================
 * Per-particle element maps.  z = (x, xp, y, yp, s, dp).
 * ====================================================================== */

/* Exact drift (Sec. 2.1 listings): x += x'L, y += y'L and the path length
 * L sqrt(1+x'^2+y'^2), here kept as the deviation from L, written
 * L u / (1 + sqrt(1+u)) with u = x'^2 + y'^2 to avoid cancellation. */
static void edrift(double *z, double L) {
  double xp = z[1], yp = z[3];
  double u = fma(xp, xp, yp * yp);
  z[0] = fma(xp, L, z[0]);
  z[2] = fma(yp, L, z[2]);
  z[4] = fma(L, u / (1.0 + sqrt(1.0 + u)), z[4]);
}

/* Second-order map in TRANSPORT form: every output from the input vector,
 * z_i = C_i + sum_j R_ij z_j + sum_{j<=k} T_ijk z_j z_k, a plain left-to-right
 * sum over the non-zero terms in the order C, R by ascending j, T by
 * ascending (j,k): the first term is the sum so far (a product of a
 * coefficient and the coordinates), each later term is added with one fma.
 * A row without terms yields 0; a row whose only term is R_ii = 1 is an
 * exact identity. */
static void map2(double *z, const double *coef) {
  double in[6], out[6];
  memcpy(in, z, sizeof in);
  for (int i = 0; i < 6; ++i) {
    double acc = 0.0;
    int have = 0;
    if (coef[i] != 0.0) {
      acc = coef[i];
      have = 1;
    }
    for (int j = 0; j < 6; ++j) {
      double r = coef[6 + i * 6 + j];
      if (r != 0.0) {
        acc = have ? fma(r, in[j], acc) : r * in[j];
        have = 1;
      }
    }
    int p = 0;
    for (int j = 0; j < 6; ++j)
      for (int k = j; k < 6; ++k, ++p) {
        double t = coef[42 + i * 21 + p];
        if (t != 0.0) {
          double m = in[j] * in[k];
          acc = have ? fma(t, m, acc) : t * m;
          have = 1;
        }
      }
    out[i] = acc;
  }
  memcpy(z, out, sizeof out);
}

/* Third-order map (the M3 matrix tracking of the element table): as map2,
 * then the cubic terms U_ijkl z_j z_k z_l, (j,k,l) ascending with
 * j <= k <= l, each monomial rounded as (z_j z_k) z_l. */
static void map3(double *z, const double *coef) {
  double in[6], out[6];
  memcpy(in, z, sizeof in);
  for (int i = 0; i < 6; ++i) {
    double acc = 0.0;
    int have = 0;
    if (coef[i] != 0.0) {
      acc = coef[i];
      have = 1;
    }
    for (int j = 0; j < 6; ++j) {
      double r = coef[6 + i * 6 + j];
      if (r != 0.0) {
        acc = have ? fma(r, in[j], acc) : r * in[j];
        have = 1;
      }
    }
    int p = 0;
    for (int j = 0; j < 6; ++j)
      for (int k = j; k < 6; ++k, ++p) {
        double tc = coef[42 + i * 21 + p];
        if (tc != 0.0) {
          double m = in[j] * in[k];
          acc = have ? fma(tc, m, acc) : tc * m;
          have = 1;
        }
      }
    int q = 0;
    for (int j = 0; j < 6; ++j)
      for (int k = j; k < 6; ++k)
        for (int l = k; l < 6; ++l, ++q) {
          double u = coef[168 + i * 56 + q];
          if (u != 0.0) {
            double m = (in[j] * in[k]) * in[l];
            acc = have ? fma(u, m, acc) : u * m;
            have = 1;
          }
        }
    out[i] = acc;
  }
  memcpy(z, out, sizeof out);
}

/* slopes -> canonical (px, py) = (1+delta)(x', y') / sqrt(1 + x'^2 + y'^2) */
static void to_canonical(const double *z, double opd, double *px, double *py) {
  double xp = z[1], yp = z[3];
  double u = fma(xp, xp, yp * yp);
  double pz = opd / sqrt(1.0 + u);
  *px = xp * pz;
  *py = yp * pz;
}
/* canonical -> slopes x' = px/pz, y' = py/pz, pz = sqrt((1+delta)^2 - px^2 - py^2) */
static void to_slopes(double *z, double opd2, double px, double py) {
  double q = fma(px, px, py * py);
  double pz = sqrt(opd2 - q);
  double r = 1.0 / pz;
  z[1] = px * r;
  z[3] = py * r;
}

/* Thin multipole of order n (KnL): Delta px - i Delta py = -(KnL/n!) (x+iy)^n,
 * a kick on the canonical momenta; x, y, s unchanged. */
static void mult(double *z, double kn, int order) {
  double opd = 1.0 + z[5];
  double opd2 = opd * opd;
  double px, py;
  to_canonical(z, opd, &px, &py);
  double x = z[0], y = z[2];
  double re = x, im = y;
  for (int m = 2; m <= order; ++m) {
    double nre = (re * x) - (im * y);
    double nim = (re * y) + (im * x);
    re = nre;
    im = nim;
  }
  px = fma(-kn, re, px);
  py = fma(kn, im, py);
  to_slopes(z, opd2, px, py);
}

/* canonical exact drift over dl (field-free Hamiltonian): x, y advance by
 * dl px/pz, dl py/pz; the path excess dl ((1+delta)/pz - 1) is written
 * cancellation-free as dl q / (pz ((1+delta) + pz)), q = px^2 + py^2.  Both
 * come from the one quotient w = dl / (pz ((1+delta) + pz)):
 * dl/pz = ((1+delta) + pz) w and the excess is q w. */
static void cdrift(double *z, double *px, double *py, double opd, double opd2, double dl) {
  double q = fma(*px, *px, *py * *py);
  double pz = sqrt(opd2 - q);
  double a = opd + pz;
  double w = dl / (pz * a);
  double t = a * w;
  z[0] = fma(*px, t, z[0]);
  z[2] = fma(*py, t, z[2]);
  z[4] = fma(q, w, z[4]);
}

typedef struct {
  int nsteps;
  double kq[4], dl[3];                       /* KQUAD */
  double kA[4], kB[4];                       /* CSBEND kicks */
  double cph[3], sph[3], vers[3], rs[3];     /* CSBEND polar drifts */
} kd_const;

static void kd_constants(const orc_elem *e, kd_const *k) {
  double c[4], d[3];
  orc_yoshida(c, d);
  k->nsteps = e->nsteps > 0 ? e->nsteps : 1;
  double ls = e->L / (double)k->nsteps;
  for (int i = 0; i < 3; ++i) k->dl[i] = d[i] * ls;
  if (e->kind == ORC_KQUAD) {
    for (int i = 0; i < 4; ++i) k->kq[i] = (c[i] * ls) * e->k;
  } else {
    double h = e->angle / e->L;
    double rho = e->L / e->angle;
    for (int i = 0; i < 4; ++i) {
      k->kA[i] = (c[i] * ls) * h;
      k->kB[i] = k->kA[i] * h;
    }
    for (int i = 0; i < 3; ++i) {
      double phi = k->dl[i] * h;
      double shalf = sin(0.5 * phi);
      k->cph[i] = cos(phi);
      k->sph[i] = sin(phi);
      k->vers[i] = 2.0 * rho * (shalf * shalf);
      k->rs[i] = rho * k->sph[i];
    }
  }
}

/* Kick-drift quadrupole (KQUAD, 4th-order symplectic integration): in
 * canonical variables, kicks Delta px = -l k1 x, Delta py = +l k1 y and exact
 * drifts between them. */
static void kquad(double *z, const kd_const *k) {
  double opd = 1.0 + z[5];
  double opd2 = opd * opd;
  double px, py;
  to_canonical(z, opd, &px, &py);
  for (int st = 0; st < k->nsteps; ++st)
    for (int i = 0; i < 4; ++i) {
      px = fma(-k->kq[i], z[0], px);
      py = fma(k->kq[i], z[2], py);
      if (i < 3) cdrift(z, &px, &py, opd, opd2, k->dl[i]);
    }
  to_slopes(z, opd2, px, py);
}

/* Canonical-kick sector bend (CSBEND): Hamiltonian -(1+hx) pz + hx + h^2x^2/2
 * split into a drift in the curved frame (a straight line, solved exactly in
 * polar coordinates over the angle phi = h dl) and the kick
 * Delta px = -l h (1 + h x). */
static void csbend(double *z, const kd_const *k) {
  double opd = 1.0 + z[5];
  double opd2 = opd * opd;
  double iopd = 1.0 / opd;
  double px, py;
  to_canonical(z, opd, &px, &py);
  for (int st = 0; st < k->nsteps; ++st)
    for (int i = 0; i < 4; ++i) {
      px = px - fma(k->kB[i], z[0], k->kA[i]);
      if (i < 3) {
        double x = z[0];
        double q = fma(px, px, py * py);
        double pz = sqrt(opd2 - q);
        double pxn = fma(px, k->cph[i], pz * k->sph[i]);
        double pzn = fma(pz, k->cph[i], -(px * k->sph[i]));
        double tau = (fma(x, k->sph[i], k->rs[i]) * opd) / pzn;
        double g = tau * iopd;
        z[0] = fma(g, pxn, fma(x, k->cph[i], -k->vers[i]));
        z[2] = fma(g, py, z[2]);
        z[4] = z[4] + (tau - k->dl[i]);
        px = pxn;
      }
    }
  to_slopes(z, opd2, px, py);
}

/* Zero-length RF cavity (RFCA): energy gain V cos(phase + k s) with the
 * reference momentum raised to P' = P + V cos(phase):
 *   delta' = (delta P + V (cos(phase + ks) - cos(phase))) / P'.
 * The cosine difference is -2 sin(a) sin(phase + a), a = ks/2, with
 * sin(phase + a) = sin(phase) cos(a) + cos(phase) sin(a) (no cancellation;
 * sin/cos of the phase are element constants), and the division by P' is a
 * multiplication by the element constant 1/P'. */
static void rfca(double *z, double hk, double sph, double cph, double volt, double pin,
                 double inv_pn) {
  double a = hk * z[4];
  double sa = orc_sin(a), ca = orc_cos(a);
  double dc = (-2.0 * fma(sph, ca, cph * sa)) * sa;
  double num = fma(z[5], pin, volt * dc);
  z[5] = num * inv_pn;
}

static int aperture_lost(const orc_elem *e, const double *z) {
  if (e->aper == ORC_APER_RECT) {
    return !(fabs(z[0]) < e->ax && fabs(z[2]) < e->ay);
  } else if (e->aper == ORC_APER_ELLIPSE) {
    double xa = z[0] * (1.0 / e->ax);
    double ya = z[2] * (1.0 / e->ay);
    double q = fma(xa, xa, ya * ya);
    return !(q < 1.0);
  }
  return 0;
}

/* ======================================================================
 * Collective primitives (Sec. 2.2 histogram, Sec. 2.3 convolution)
 * ====================================================================== */

/* range = [min s, max s] over alive particles; half-open bins of width
 * (smax - smin)/nbins, the last edge folded into the last bin; a zero
 * range puts every particle into bin 0. */
void orc_histogram(const double *s, const int64_t *lost_at, int64_t n, int32_t nbins,
                   double range[2], uint32_t *counts) {
  double smin = INFINITY, smax = -INFINITY;
  int64_t nal = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (lost_at[i] >= 0) continue;
    ++nal;
    if (s[i] < smin) smin = s[i];
    if (s[i] > smax) smax = s[i];
  }
  for (int32_t b = 0; b < nbins; ++b) counts[b] = 0;
  if (nal == 0) {
    range[0] = 0.0;
    range[1] = 0.0;
    return;
  }
  range[0] = smin;
  range[1] = smax;
  double width = smax - smin;
  double inv = width > 0.0 ? (double)nbins / width : 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (lost_at[i] >= 0) continue;
    double f = (s[i] - smin) * inv;
    if (!(f >= 0.0)) continue; /* NaN s is not binned */
    int64_t b = (int64_t)floor(f);
    if (b > nbins - 1) b = nbins - 1;
    counts[b] += 1u;
  }
}

/* Normalised resonator wake W(tau)/A = exp(-tau/tau0) cos(omega tau) on the
 * bin lags tau = m (smax - smin)/(nbins c); the m = 0 entry is W(0)/2 (a
 * particle sees half of its own wake). */
void orc_wake_table(double smin, double smax, int32_t nbins, double tau0, double omega,
                    double *w) {
  double width = smax - smin;
  double delta = width > 0.0 ? width / (double)nbins : 0.0;
  double dt = delta / C_LIGHT;
  w[0] = 0.5;
  for (int32_t m = 1; m < nbins; ++m) {
    double t = (double)m * dt;
    w[m] = orc_exp(-(t / tau0)) * orc_cos(omega * t);
  }
}

/* causal convolution V[i] = sum_{j<=i} c_j W[i-j], j ascending */
void orc_convolve(const uint32_t *counts, const double *w, int32_t nbins, double *v) {
  for (int32_t i = 0; i < nbins; ++i) {
    double acc = 0.0;
    for (int32_t j = 0; j <= i; ++j) acc = fma((double)counts[j], w[i - j], acc);
    v[i] = acc;
  }
}

/* energy kick delta -= kfac V(s), V linearly interpolated between bin
 * centres and held constant beyond the first and last centre */
static double interp_v(double s, double smin, double inv, const double *v, int32_t nbins) {
  double f = (s - smin) * inv - 0.5;
  double fl = floor(f);
  int64_t i0;
  if (!(fl >= 0.0))
    i0 = 0;
  else if (fl > (double)(nbins - 2))
    i0 = nbins - 2;
  else
    i0 = (int64_t)fl;
  double w = f - (double)i0;
  if (!(w >= 0.0)) w = 0.0;
  if (w > 1.0) w = 1.0;
  return fma(w, v[i0 + 1] - v[i0], v[i0]);
}

void orc_wake_kick(orc_beam *b, const double range[2], const double *v, int32_t nbins,
                   double kfac) {
  double width = range[1] - range[0];
  double inv = width > 0.0 ? (double)nbins / width : 0.0;
  double nk = -kfac;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < b->n; ++i) {
    if (b->lost_at[i] >= 0) continue;
    double vs = interp_v(b->z[4][i], range[0], inv, v, nbins);
    b->z[5][i] = fma(nk, vs, b->z[5][i]);
  }
}

/* ======================================================================
 * Transverse wake (the TRWAKE element of the element table; the transverse
 * part of RFCW)
 * ====================================================================== */

/* A coordinate as an integer multiple of 2^-40 m: clamped to [-1, 1] m,
 * rounded to the nearest multiple (ties to even); a NaN counts as 0. */
int64_t orc_dipole_quantum(double x) {
  if (x != x) return 0;
  if (x > 1.0) x = 1.0;
  if (x < -1.0) x = -1.0;
  return (int64_t)nearbyint(x * 0x1p40);
}

/* The histogram of s (same range, bins and counts as orc_histogram) and, per
 * bin, the sums of the quantised x and y of its particles, added as 64-bit
 * two's-complement integers (modulo 2^64): exact, whatever the order. */
void orc_dipole_histogram(const double *s, const double *x, const double *y,
                          const int64_t *lost_at, int64_t n, int32_t nbins, double range[2],
                          uint32_t *counts, int64_t *dx, int64_t *dy) {
  orc_histogram(s, lost_at, n, nbins, range, counts);
  for (int32_t b = 0; b < nbins; ++b) {
    dx[b] = 0;
    dy[b] = 0;
  }
  double width = range[1] - range[0];
  double inv = width > 0.0 ? (double)nbins / width : 0.0;
  for (int64_t i = 0; i < n; ++i) {
    if (lost_at[i] >= 0) continue;
    double f = (s[i] - range[0]) * inv;
    if (!(f >= 0.0)) continue;
    int64_t b = (int64_t)floor(f);
    if (b > nbins - 1) b = nbins - 1;
    dx[b] = (int64_t)((uint64_t)dx[b] + (uint64_t)orc_dipole_quantum(x[i]));
    dy[b] = (int64_t)((uint64_t)dy[b] + (uint64_t)orc_dipole_quantum(y[i]));
  }
}

/* dipole sums in metres: one rounding of the integer, then an exact scaling */
void orc_dipole_metres(const int64_t *d, int32_t nbins, double *out) {
  for (int32_t b = 0; b < nbins; ++b) out[b] = (double)d[b] * 0x1p-40;
}

/* Normalised transverse resonator wake W(tau)/A = exp(-tau/tau0) sin(omega
 * tau) on the bin lags tau = m (smax - smin)/(nbins c); zero at m = 0. */
void orc_trwake_table(double smin, double smax, int32_t nbins, double tau0, double omega,
                      double *w) {
  double width = smax - smin;
  double delta = width > 0.0 ? width / (double)nbins : 0.0;
  double dt = delta / C_LIGHT;
  w[0] = 0.0;
  for (int32_t m = 1; m < nbins; ++m) {
    double t = (double)m * dt;
    w[m] = orc_exp(-(t / tau0)) * orc_sin(omega * t);
  }
}

/* causal convolution of binary64 weights, V[i] = sum_{j<=i} c_j W[i-j], j ascending */
void orc_convolve_f64(const double *c, const double *w, int32_t nbins, double *v) {
  for (int32_t i = 0; i < nbins; ++i) {
    double acc = 0.0;
    for (int32_t j = 0; j <= i; ++j) acc = fma(c[j], w[i - j], acc);
    v[i] = acc;
  }
}

/* transverse kick: the canonical momenta gain kfac V_x(s), kfac V_y(s), with
 * V interpolated as for the energy kick; slopes are converted to canonical
 * momenta and back as in the thin multipole */
void orc_trwake_kick(orc_beam *b, const double range[2], const double *vx, const double *vy,
                     int32_t nbins, double kfac) {
  double width = range[1] - range[0];
  double inv = width > 0.0 ? (double)nbins / width : 0.0;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < b->n; ++i) {
    if (b->lost_at[i] >= 0) continue;
    double z[6];
    for (int k = 0; k < 6; ++k) z[k] = b->z[k][i];
    double ux = interp_v(z[4], range[0], inv, vx, nbins);
    double uy = interp_v(z[4], range[0], inv, vy, nbins);
    double opd = 1.0 + z[5];
    double px, py;
    to_canonical(z, opd, &px, &py);
    px = fma(kfac, ux, px);
    py = fma(kfac, uy, py);
    to_slopes(z, opd * opd, px, py);
    b->z[1][i] = z[1];
    b->z[3][i] = z[3];
  }
}

/* Neumaier-compensated sum of an array */
static double csum(const double *a, int64_t n) {
  double s = 0.0, c = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double t = s + a[i];
    if (fabs(s) >= fabs(a[i]))
      c += (s - t) + a[i];
    else
      c += (a[i] - t) + s;
    s = t;
  }
  return s + c;
}

/* Beam moments over alive particles (the centroid and second-moment
 * reductions of Sec. 2.4): n, the six means and the 21 central second
 * moments (population normalisation), two passes with compensated sums.
 * With no particle alive every entry is 0 (the paper defines no moments of
 * an empty beam; 0 stands in for the undefined 0/0). */
void orc_moments(const orc_beam *b, double out[28]) {
  int64_t nal = 0;
  for (int64_t i = 0; i < b->n; ++i)
    if (b->lost_at[i] < 0) ++nal;
  if (nal == 0) {
    for (int k = 0; k < 28; ++k) out[k] = 0.0;
    return;
  }
  double *buf = (double *)malloc((size_t)(nal > 0 ? nal : 1) * sizeof(double));
  double mean[6];
  out[0] = (double)nal;
  for (int k = 0; k < 6; ++k) {
    int64_t m = 0;
    for (int64_t i = 0; i < b->n; ++i)
      if (b->lost_at[i] < 0) buf[m++] = b->z[k][i];
    mean[k] = csum(buf, nal) / (double)nal;
    out[1 + k] = mean[k];
  }
  int o = 7;
  for (int k = 0; k < 6; ++k)
    for (int l = k; l < 6; ++l) {
      int64_t m = 0;
      for (int64_t i = 0; i < b->n; ++i)
        if (b->lost_at[i] < 0) buf[m++] = (b->z[k][i] - mean[k]) * (b->z[l][i] - mean[l]);
      out[o++] = csum(buf, nal) / (double)nal;
    }
  free(buf);
}

/* Loss reordering (the role of the paper's loss algorithm, Sec. 2.5, with a
 * stable order): alive particles first in their current order, then the
 * lost ones by loss record descending (latest loss first), ties in current
 * order.  Returns the number alive. */
static const int64_t *g_keys;
static int cmp_lost(const void *a, const void *b) {
  int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
  int64_t ka = g_keys[ia], kb = g_keys[ib];
  int aa = ka < 0, ab = kb < 0;
  if (aa != ab) return aa ? -1 : 1;      /* alive first */
  if (!aa && ka != kb) return ka > kb ? -1 : 1; /* later loss first */
  return ia < ib ? -1 : (ia > ib ? 1 : 0);
}
int64_t orc_compact(orc_beam *b) {
  int64_t n = b->n;
  int64_t *perm = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  g_keys = b->lost_at;
  qsort(perm, (size_t)n, sizeof(int64_t), cmp_lost);
  double *tmp = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
  for (int k = 0; k < 6; ++k) {
    for (int64_t i = 0; i < n; ++i) tmp[i] = b->z[k][perm[i]];
    memcpy(b->z[k], tmp, (size_t)n * sizeof(double));
  }
  uint32_t *tid = (uint32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(uint32_t));
  int64_t *tla = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  int64_t nal = 0;
  for (int64_t i = 0; i < n; ++i) {
    tid[i] = b->id[perm[i]];
    tla[i] = b->lost_at[perm[i]];
    if (tla[i] < 0) ++nal;
  }
  memcpy(b->id, tid, (size_t)n * sizeof(uint32_t));
  memcpy(b->lost_at, tla, (size_t)n * sizeof(int64_t));
  free(perm);
  free(tmp);
  free(tid);
  free(tla);
  return nal;
}

/* ======================================================================
 * Tracking driver
 * ====================================================================== */
int64_t orc_track(orc_beam *b, const orc_elem *lat, int32_t nelem, int32_t passes,
                  int32_t first_pass, double p_ref, uint64_t seed, double *moments) {
  double P = p_ref;
  int64_t n = b->n;
  kd_const *kd = (kd_const *)calloc((size_t)(nelem > 0 ? nelem : 1), sizeof(kd_const));
  for (int32_t e = 0; e < nelem; ++e)
    if (lat[e].kind == ORC_KQUAD || lat[e].kind == ORC_CSBEND) kd_constants(&lat[e], &kd[e]);
  double *qcoef = (double *)calloc((size_t)(nelem > 0 ? nelem : 1) * 504, sizeof(double));
  for (int32_t e = 0; e < nelem; ++e) {
    if (lat[e].kind == ORC_QUAD && lat[e].order == 3)
      orc_quad3_coef(lat[e].L, lat[e].k, qcoef + 504 * e);
    else if (lat[e].kind == ORC_QUAD)
      orc_quad_coef(lat[e].L, lat[e].k, qcoef + 504 * e);
    if (lat[e].kind == ORC_MAP2) memcpy(qcoef + 504 * e, lat[e].coef, 168 * sizeof(double));
    if (lat[e].kind == ORC_MAP3) memcpy(qcoef + 504 * e, lat[e].coef, 504 * sizeof(double));
  }
  for (int32_t p = 0; p < passes; ++p) {
    int64_t gp = (int64_t)first_pass + p;
    for (int32_t e = 0; e < nelem; ++e) {
      const orc_elem *el = &lat[e];
      if (el->kind == ORC_WAKE) {
        int32_t nb = el->nbins;
        uint32_t *counts = (uint32_t *)malloc((size_t)nb * sizeof(uint32_t));
        double *w = (double *)malloc((size_t)nb * sizeof(double));
        double *v = (double *)malloc((size_t)nb * sizeof(double));
        double range[2];
        orc_histogram(b->z[4], b->lost_at, n, nb, range, counts);
        orc_wake_table(range[0], range[1], nb, el->wake_tau0, el->wake_omega, w);
        orc_convolve(counts, w, nb, v);
        double kfac = ((el->charge / (double)b->n0) * el->wake_A) / P;
        orc_wake_kick(b, range, v, nb, kfac);
        free(counts);
        free(w);
        free(v);
      }
      if (el->kind == ORC_TRWAKE) {
        int32_t nb = el->nbins;
        uint32_t *counts = (uint32_t *)malloc((size_t)nb * sizeof(uint32_t));
        int64_t *dq = (int64_t *)malloc((size_t)nb * 2 * sizeof(int64_t));
        double *dm = (double *)malloc((size_t)nb * 2 * sizeof(double));
        double *w = (double *)malloc((size_t)nb * sizeof(double));
        double *v = (double *)malloc((size_t)nb * 2 * sizeof(double));
        double range[2];
        orc_dipole_histogram(b->z[4], b->z[0], b->z[2], b->lost_at, n, nb, range, counts, dq,
                             dq + nb);
        orc_dipole_metres(dq, 2 * nb, dm);
        orc_trwake_table(range[0], range[1], nb, el->wake_tau0, el->wake_omega, w);
        orc_convolve_f64(dm, w, nb, v);
        orc_convolve_f64(dm + nb, w, nb, v + nb);
        double kfac = ((el->charge / (double)b->n0) * el->wake_A) / P;
        orc_trwake_kick(b, range, v, v + nb, nb, kfac);
        free(counts);
        free(dq);
        free(dm);
        free(w);
        free(v);
      }
      double pin = P, pn = P, hk = 0.0, sph = 0.0, cph = 0.0, inv_pn = 0.0;
      if (el->kind == ORC_RFCA) {
        sph = sin(el->phase);
        cph = cos(el->phase);
        pn = P + el->volt * cph;
        inv_pn = 1.0 / pn;
        hk = 0.5 * ((TWO_PI * el->freq) / C_LIGHT);
      }
      double kn = 0.0;
      if (el->kind == ORC_MULT) kn = el->k / fact(el->order);
      int64_t rec = (int64_t)(((uint64_t)gp << 32) | (uint32_t)e);
#pragma omp parallel for schedule(static)
      for (int64_t i = 0; i < n; ++i) {
        if (b->lost_at[i] >= 0) continue;
        double z[6];
        for (int k = 0; k < 6; ++k) z[k] = b->z[k][i];
        switch (el->kind) {
          case ORC_EDRIFT: edrift(z, el->L); break;
          case ORC_QUAD:
            if (el->order == 3)
              map3(z, qcoef + 504 * e);
            else
              map2(z, qcoef + 504 * e);
            break;
          case ORC_MAP2: map2(z, qcoef + 504 * e); break;
          case ORC_MAP3: map3(z, qcoef + 504 * e); break;
          case ORC_MULT: mult(z, kn, el->order); break;
          case ORC_KQUAD: kquad(z, &kd[e]); break;
          case ORC_CSBEND: csbend(z, &kd[e]); break;
          case ORC_RFCA: rfca(z, hk, sph, cph, el->volt, pin, inv_pn); break;
          case ORC_RADKICK:
            z[5] = fma(el->sigma, orc_gauss(b->id[i], (uint32_t)gp, ORC_TAG_RAD, seed), z[5]);
            break;
          default: break;
        }
        for (int k = 0; k < 6; ++k) b->z[k][i] = z[k];
        if (aperture_lost(el, z)) b->lost_at[i] = rec;
      }
      if (el->kind == ORC_RFCA) P = pn;
    }
    if (moments) orc_moments(b, moments + 28 * (size_t)p);
  }
  free(kd);
  free(qcoef);
  return orc_compact(b);
}

void orc_set_threads(int32_t n) {
#ifdef _OPENMP
  omp_set_num_threads(n);
#else
  (void)n;
#endif
}
int32_t orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
