/* trk.h -- C-ABI of the MI355X lumped-element particle tracker (libtrk.so).
 *
 * The library pushes N particles of 6D binary64 phase space through a
 * beamline element by element (the problem statement of King et al.,
 * "GPU acceleration and performance of the particle-beam-dynamics code
 * Elegant", Sec. 1-2), on one AMD Instinct MI355X (gfx950), with hand-written
 * HIP kernels.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Coordinates: x [m], x' = dx/ds, y [m], y' = dy/ds, s [m] = path-length
 *   deviation from the reference particle (positive = behind), delta =
 *   (p - p0)/p0.  The slope form follows the paper's exact-drift listings
 *   (Sec. 2.1); s is kept as a deviation so that its precision does not
 *   decay with the distance travelled.
 * Layout: structure of arrays (Sec. 2: SoA for coalesced access), one
 *   contiguous binary64 array per coordinate.  Device pointers only.
 * Alive set: particle i is alive iff i < *n_alive.  Every call that can lose
 *   particles reorders the arrays before it returns so that this holds
 *   (alive ones first, in their previous order; lost ones after, latest loss
 *   first) -- the role of the paper's particle-loss algorithm (Sec. 2.5),
 *   made stable.  lost_at[i] = -1 for alive particles, else
 *   (pass << 32) | element_index of the element at whose exit the particle
 *   failed the aperture; its coordinates are frozen at that exit.
 * Ownership: beams, outputs and workspaces are allocated by the caller
 *   (e.g. as torch tensors); the library never frees them.  A lattice handle
 *   owns a device copy of its element records.
 * Streams: every call is asynchronous on the given hipStream_t (passed as
 *   void*; NULL is the null stream) and does not synchronise the host.
 *   Calls on one workspace must be serialised (same stream or events).
 * Errors: every function returns TRK_OK (0) or a negative status; no C++
 *   exception crosses the ABI.  trk_last_error() gives a message for the
 *   calling thread.  Invalid sizes and host pointers passed where device
 *   pointers are required are rejected before anything is launched (the
 *   analog of the paper's host-pointer nullification, Sec. 5.1).
 *   Asynchronous device faults surface at the next synchronising HIP call.
 */
#ifndef TRK_H
#define TRK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define TRK_OK 0
#define TRK_EINVAL (-1) /* invalid argument or lattice */
#define TRK_EPTR (-2)   /* a host pointer where a device pointer is required */
#define TRK_EHIP (-3)   /* HIP runtime error */
#define TRK_ENOMEM (-4) /* device allocation failed */
#define TRK_ERANGE (-5) /* a size beyond a documented limit (workspace, bins) */

/* ------------------------------------------------------------------ elements
 * Element kinds (the beamline elements of the paper's element table, Sec. 3):
 *   TRK_EDRIFT  exact drift, length L (Sec. 2.1 listings).
 *   TRK_QUAD    thick quadrupole L, K1 as a second-order transfer matrix.
 *   TRK_MAP2    explicit second-order map: coef = C[6], R[6][6], T[6][21].
 *   TRK_MULT    thin multipole, order n (1 quad, 2 sext, 3 oct), k = KnL.
 *   TRK_KQUAD   kick-drift quadrupole L, K1, nsteps 4th-order symplectic steps.
 *   TRK_CSBEND  canonical-kick sector bend L, angle, nsteps steps.
 *   TRK_RFCA    zero-length RF cavity: volt [V], phase [rad], freq [Hz].
 *   TRK_WAKE    longitudinal wake: histogram of s into nbins bins, causal
 *               convolution with W(t) = A exp(-t/tau0) cos(omega t), energy
 *               kick; charge = bunch charge [C] (Sec. 2.2-2.3).
 *   TRK_RADKICK random energy kick delta += sigma g, g ~ N(0,1) from
 *               Philox4x32-10 with counter (id, pass, 2, 0), key = seed.
 *   TRK_MARKER  nothing (carries an aperture only).
 * Any element may carry an aperture checked at its exit:
 *   TRK_APER_RECT     survive iff |x| < ax and |y| < ay;
 *   TRK_APER_ELLIPSE  survive iff (x/ax)^2 + (y/ay)^2 < 1.
 * A non-finite x or y fails every aperture. */
enum trk_kind {
  TRK_EDRIFT = 1, TRK_QUAD = 2, TRK_MAP2 = 3, TRK_MULT = 4, TRK_KQUAD = 5,
  TRK_CSBEND = 6, TRK_RFCA = 7, TRK_WAKE = 8, TRK_RADKICK = 9, TRK_MARKER = 10
};
enum trk_aperture { TRK_APER_NONE = 0, TRK_APER_RECT = 1, TRK_APER_ELLIPSE = 2 };
enum trk_wake_mode { TRK_WAKE_FP64 = 0, TRK_WAKE_FP32_MFMA = 1 };

typedef struct trk_element {
  int32_t kind;      /* enum trk_kind */
  int32_t aperture;  /* enum trk_aperture */
  int32_t order;     /* TRK_MULT order, 1..8 */
  int32_t nsteps;    /* TRK_KQUAD/TRK_CSBEND integration steps, >= 1 */
  int32_t nbins;     /* TRK_WAKE bins, 2..TRK_MAX_BINS */
  int32_t reserved;
  double L, k, angle;
  double volt, phase, freq;
  double wake_A, wake_tau0, wake_omega, charge;
  double sigma;
  double ax, ay;
  const double *coef; /* TRK_MAP2: 168 host doubles, copied at creation */
} trk_element;

#define TRK_MAX_BINS 4096
#define TRK_MAX_ELEMENTS 65536

/* ------------------------------------------------------------------ beam */
typedef struct trk_beam {
  double *x, *xp, *y, *yp, *s, *dp; /* device [n_total] each */
  uint32_t *id;                     /* device [n_total]: particle identity */
  int64_t *lost_at;                 /* device [n_total] */
  int64_t *n_alive;                 /* device scalar */
  int64_t n_total;                  /* host value: array length, also the
                                       macro-particle count N0 (charge Q/N0) */
} trk_beam;

/* ------------------------------------------------------------------ lattice
 * Copies the records to a library-owned device buffer, checks them and
 * precomputes every per-element constant (transfer-map coefficients,
 * integrator constants).  Immutable afterwards; usable from any stream. */
typedef struct trk_lattice trk_lattice;
int trk_lattice_create(const trk_element *elems, int32_t n, trk_lattice **out);
void trk_lattice_destroy(trk_lattice *lat);

/* ------------------------------------------------------------------ options */
typedef struct trk_opts {
  uint64_t seed;                /* Philox key for TRK_RADKICK */
  int32_t first_pass;           /* global index of the first pass (loss records, RNG) */
  int32_t passes_per_launch;    /* fusion depth in passes when the lattice has no
                                   TRK_WAKE (0 = 16) */
  int32_t max_elems_per_launch; /* fusion depth in elements (0 = no limit) */
  int32_t wake_mode;            /* enum trk_wake_mode */
  int32_t run_ppt;              /* launch shape of the fused runs (0 = automatic):
                                   particles per thread, 1, 2, 4 or 8 */
  int32_t run_blocks;           /* grid cap of grid-stride runs (0 = automatic) */
  int32_t run_longit;           /* runs touching only s and delta: 0 automatic
                                   (two-coordinate kernel), -1 generic kernel */
  int32_t reserved;
  double p_ref_eV;              /* reference momentum at the entry of the first
                                   pass [eV/c]; raised by V cos(phase) per RFCA */
  double *moments;              /* NULL or device [passes][28]: per pass, after its
                                   last element: n, mean[6], central second
                                   moments upper triangle row-major [21] */
} trk_opts;

/* Device workspace needed by trk_track and the collective calls for a beam of
 * n_total particles on this lattice (lat may be NULL for the standalone
 * collective calls).  The caller allocates it; contents need no
 * initialisation and are clobbered by every call. */
size_t trk_workspace_size(const trk_lattice *lat, int64_t n_total);

/* track(beam, lattice, passes): `passes` passes through the lattice.  Runs of
 * consecutive elements are fused into one kernel (coordinates loaded once,
 * kept in registers, stored once); TRK_WAKE splits runs.  Results do not
 * depend on the fusion depth.  Returns after enqueuing; the beam is
 * reordered (alive set first) when the last kernel completes. */
int trk_track(trk_beam *beam, const trk_lattice *lat, int32_t passes, const trk_opts *opts,
              void *workspace, size_t workspace_bytes, void *stream);

/* histogram (Sec. 2.2): range_dev[2] = (min s, max s) over alive particles
 * ((0, 0) if none); counts_dev[nbins] = particles per half-open bin of width
 * (max - min)/nbins, the upper edge folded into the last bin; all in bin 0
 * if min == max.  2 <= nbins <= TRK_MAX_BINS. */
int trk_histogram(const trk_beam *beam, int32_t nbins, double *range_dev, uint32_t *counts_dev,
                  void *workspace, size_t workspace_bytes, void *stream);

/* wake convolution (Sec. 2.3): v_dev[i] = sum_{j<=i} counts[j] W~[i-j] with
 * W~[0] = 1/2 and W~[m] = exp(-t_m/tau0) cos(omega t_m), t_m = m (max-min)/
 * (nbins c).  TRK_WAKE_FP64 sums j ascending with binary64 fma (bit-exact
 * with the oracle); TRK_WAKE_FP32_MFMA rounds W~ and the counts to binary32
 * and sums with FP32 matrix-core accumulation (counts must be < 2^24). */
int trk_wake_convolve(const uint32_t *counts_dev, int32_t nbins, const double *range_dev,
                      double tau0, double omega, int32_t mode, double *v_dev, void *stream);

/* wake_kick: the convolution above followed by the energy kick
 * delta -= kfac V(s) on alive particles, V linearly interpolated between bin
 * centres and held beyond the outer centres, kfac = ((charge/N0) A)/p_ref_eV. */
typedef struct trk_wake {
  double A, tau0, omega, charge;
} trk_wake;
int trk_wake_kick(trk_beam *beam, const uint32_t *counts_dev, int32_t nbins,
                  const double *range_dev, const trk_wake *w, double p_ref_eV, int32_t mode,
                  void *workspace, size_t workspace_bytes, void *stream);

/* moments (Sec. 2.4 reductions): out_dev[28] = n, mean[6], central second
 * moments [21] (population normalisation) over alive particles, two passes,
 * fixed-order binary64 trees (deterministic for a given n_total). */
int trk_moments(const trk_beam *beam, double *out_dev, void *workspace, size_t workspace_bytes,
                void *stream);

/* compact_lost (Sec. 2.5): particles in [0, *n_alive) with lost_at >= 0 move
 * behind the survivors, ordered by lost_at descending, ties in their previous
 * order; survivors keep their order; *n_alive is decreased.  Particles at
 * and beyond the old *n_alive are not touched.  Done on the device
 * (scan, single-workgroup stable radix sort of the lost subset by a dense
 * rank of (pass, element), scatter), so the host never waits. */
int trk_compact_lost(trk_beam *beam, void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------ batches
 * Many variants of one lattice structure (same element kinds in the same
 * order; strengths, apertures and seeds may differ), each with its own beam
 * of uneven size, tracked in one persistent launch: work is split into
 * (variant, chunk) tickets that a grid of a few blocks per compute unit pulls
 * from an atomic counter.  Every particle's result equals that of its
 * variant tracked alone with trk_track (same element arithmetic, random
 * kicks keyed by (id, pass) with the variant's seed).  Particles stay in
 * place (no reordering); lost ones get their lost_at record.  RF cavities
 * and wakes are not supported in batches.
 *
 * trk_batch_create: lats[nvar] lattices; seg_off[nvar+1] host offsets of the
 * variants' segments in the concatenated beam (seg_off[0] = 0); seeds[nvar].
 * Copies everything to a library-owned handle. */
typedef struct trk_batch trk_batch;
int trk_batch_create(const trk_lattice *const *lats, int32_t nvar, const int64_t *seg_off,
                     const uint64_t *seeds, trk_batch **out);
void trk_batch_destroy(trk_batch *b);

/* Launch schedule (the autotuner's search space): ppt particles per thread
 * (1, 2 or 4), blocks_per_cu persistent blocks per compute unit,
 * passes_per_launch passes per persistent launch (0 = all), use_graph: 1 to
 * capture the launch sequence in a hipGraph (captured on a stream the handle
 * owns, cached on the handle, replayed on the caller's stream while the
 * arguments repeat; a handle must not be used from two threads at once). */
typedef struct trk_batch_tuning {
  int32_t ppt, blocks_per_cu, passes_per_launch, use_graph;
} trk_batch_tuning;

/* workspace for moments of up to passes_per_launch passes per launch
 * (64 at most) */
size_t trk_batch_workspace_size(const trk_batch *b, int32_t passes_per_launch);

/* beam: the concatenated beam (n_total = seg_off[nvar]; n_alive unused);
 * moments_dev: NULL or [nvar][passes][28] (as trk_opts.moments, unshifted
 * one-pass sums). */
int trk_track_batched(trk_batch *b, const trk_beam *beam, int32_t passes, int32_t first_pass,
                      const trk_batch_tuning *tune, double *moments_dev, void *workspace,
                      size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------ test hooks
 * Bit-exactness probes of the device arithmetic used by the kernels.
 * fn: 0 sin, 1 cos, 2 log, 3 exp (own implementations), 4 sqrt, 5 x / y. */
int trk_elementary(int32_t fn, const double *x_dev, const double *y_dev, double *out_dev,
                   int64_t n, void *stream);
/* Philox4x32-10 blocks: ctr_dev[n][4], key_dev[n][2] -> out_dev[n][4]. */
int trk_philox4x32_10(const uint32_t *ctr_dev, const uint32_t *key_dev, uint32_t *out_dev,
                      int64_t n, void *stream);
/* standard normals g(id[i], step, tag, seed) as used by TRK_RADKICK */
int trk_gauss(const uint32_t *id_dev, uint32_t step, uint32_t tag, uint64_t seed,
              double *out_dev, int64_t n, void *stream);

/* ------------------------------------------------------------------ misc */
const char *trk_status_string(int status);
const char *trk_last_error(void);
/* per-kernel-class device time (ms) and launch count accumulated with HIP
 * events while enabled; class 0 = fused element run. */
int trk_profile_enable(int32_t on);
int trk_profile_read(int32_t kernel_class, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif
