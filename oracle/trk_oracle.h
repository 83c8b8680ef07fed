/* trk_oracle.h -- plain CPU oracle of lumped-element particle tracking.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP path: both are written independently from the same written
 * arithmetic specification (the evaluation order and fma positions of every
 * element formula), which is what makes bit-equality a meaningful check.
 *
 * Coordinates are (x, x', y, y', s, delta): slopes as in the paper's exact
 * drift listing (Sec. 2.1), s the path-length deviation from the reference
 * particle, delta = (p - p0)/p0.  All arithmetic is IEEE binary64 with
 * floating-point contraction disabled; fma appears only where written.
 */
#ifndef TRK_ORACLE_H
#define TRK_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_EDRIFT = 1, ORC_QUAD = 2, ORC_MAP2 = 3, ORC_MULT = 4, ORC_KQUAD = 5,
  ORC_CSBEND = 6, ORC_RFCA = 7, ORC_WAKE = 8, ORC_RADKICK = 9, ORC_MARKER = 10,
  ORC_TRWAKE = 11, ORC_MAP3 = 12
};
enum { ORC_APER_NONE = 0, ORC_APER_RECT = 1, ORC_APER_ELLIPSE = 2 };
enum { ORC_TAG_RAD = 2 };

typedef struct orc_elem {
  int32_t kind, aper, order, nsteps, nbins, pad;
  double L, k, angle;
  double volt, phase, freq;
  double wake_A, wake_tau0, wake_omega, charge;
  double sigma;
  double ax, ay;
  double coef[504]; /* MAP2: C[6], R[6][6], T[6][21] (pairs j<=k row-major);
                       MAP3: then U[6][56] (triples j<=k<=l, lexicographic);
                       QUAD: order 3 selects the third-order map */
} orc_elem;

typedef struct orc_beam {
  double *z[6];        /* x, xp, y, yp, s, dp; each [n] */
  uint32_t *id;        /* [n] */
  int64_t *lost_at;    /* [n]; -1 alive, else (pass << 32) | element */
  int64_t n;           /* array length */
  int64_t n0;          /* macro-particle count defining the charge per particle */
} orc_beam;

/* own elementary functions (Cody-Waite reduction + fixed polynomials) */
double orc_sin(double x);
double orc_cos(double x);
double orc_log(double x);
double orc_exp(double x);

/* Philox4x32-10 (Salmon et al., SC'11) and the Box-Muller normal */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_gauss(uint32_t id, uint32_t step, uint32_t tag, uint64_t seed);

/* second-order thick-quad map coefficients (168 doubles) */
void orc_quad_coef(double L, double k1, double coef[168]);
/* third-order thick-quad map coefficients (504 doubles) */
void orc_quad3_coef(double L, double k1, double coef[504]);
/* Yoshida-4 coefficients c[4], d[3] */
void orc_yoshida(double c[4], double d[3]);

/* tracking: returns the number of alive particles after the final reorder.
 * moments: NULL or [passes][28] (n, mean[6], central second moments [21]). */
int64_t orc_track(orc_beam *b, const orc_elem *lat, int32_t nelem, int32_t passes,
                  int32_t first_pass, double p_ref, uint64_t seed, double *moments);

/* collective primitives */
void orc_histogram(const double *s, const int64_t *lost_at, int64_t n, int32_t nbins,
                   double range[2], uint32_t *counts);
void orc_wake_table(double smin, double smax, int32_t nbins, double tau0, double omega,
                    double *w);
void orc_convolve(const uint32_t *counts, const double *w, int32_t nbins, double *v);
void orc_wake_kick(orc_beam *b, const double range[2], const double *v, int32_t nbins,
                   double kfac);
/* transverse wake: dipole sums of x and y per bin in units of 2^-40 m
 * (exact 64-bit integers), the sine resonator table, the binary64
 * convolution and the kick of the canonical transverse momenta */
int64_t orc_dipole_quantum(double x);
void orc_dipole_histogram(const double *s, const double *x, const double *y,
                          const int64_t *lost_at, int64_t n, int32_t nbins, double range[2],
                          uint32_t *counts, int64_t *dx, int64_t *dy);
void orc_dipole_metres(const int64_t *d, int32_t nbins, double *out);
void orc_trwake_table(double smin, double smax, int32_t nbins, double tau0, double omega,
                      double *w);
void orc_convolve_f64(const double *c, const double *w, int32_t nbins, double *v);
void orc_trwake_kick(orc_beam *b, const double range[2], const double *vx, const double *vy,
                     int32_t nbins, double kfac);
void orc_moments(const orc_beam *b, double out[28]);
int64_t orc_compact(orc_beam *b);

void orc_set_threads(int32_t n);
int32_t orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
