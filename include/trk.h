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
 * Alive set: particle i is alive iff i < *n_alive (a value above n_total
 *   counts as n_total, and a compaction stores the clamped count back).
 *   Every call that can lose particles reorders the arrays before it returns
 *   so that this holds (alive ones first, in their previous order; lost
 *   ones after, latest loss first) -- the role of the paper's
 *   particle-loss algorithm (Sec. 2.5), made stable.  lost_at[i] = -1 for
 *   alive particles, else (pass << 32) | element_index of the element at
 *   whose exit the particle failed the aperture; its coordinates are frozen
 *   at that exit.
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
 *   TRK_QUAD    thick quadrupole L, K1 as a second-order transfer matrix
 *               (order 3: third order, the model's chromatic cubic terms).
 *   TRK_MAP2    explicit second-order map: coef = C[6], R[6][6], T[6][21].
 *   TRK_MAP3    explicit third-order map (the M3 matrix tracking): coef =
 *               C, R, T as MAP2, then U[6][56] over the monomials z_j z_k z_l,
 *               j <= k <= l in lexicographic order.
 *   TRK_MULT    thin multipole, order n (1 quad, 2 sext, 3 oct), k = KnL.
 *   TRK_KQUAD   kick-drift quadrupole L, K1, nsteps 4th-order symplectic steps.
 *   TRK_CSBEND  canonical-kick sector bend L, angle, nsteps steps.
 *   TRK_RFCA    zero-length RF cavity: volt [V], phase [rad], freq [Hz].
 *   TRK_WAKE    longitudinal wake: histogram of s into nbins bins, causal
 *               convolution with W(t) = A exp(-t/tau0) cos(omega t), energy
 *               kick; charge = bunch charge [C] (Sec. 2.2-2.3).
 *   TRK_TRWAKE  transverse wake (the transverse part of the RF cavity with
 *               wakes in the element table): the histogram of s with, per
 *               bin, the sums of x and y; their causal convolution with
 *               W(t) = A exp(-t/tau0) sin(omega t), A in V/(C m); a kick of
 *               the canonical transverse momenta (see trk_trwake_kick).
 *   TRK_RADKICK random energy kick delta += sigma g, g ~ N(0,1) from
 *               Philox4x32-10 with counter (id, pass, 2, 0), key = seed.
 *   TRK_MARKER  nothing (carries an aperture only).
 * Any element may carry an aperture checked at its exit:
 *   TRK_APER_RECT     survive iff |x| < ax and |y| < ay;
 *   TRK_APER_ELLIPSE  survive iff (x/ax)^2 + (y/ay)^2 < 1.
 * A non-finite x or y fails every aperture. */
enum trk_kind {
  TRK_EDRIFT = 1, TRK_QUAD = 2, TRK_MAP2 = 3, TRK_MULT = 4, TRK_KQUAD = 5,
  TRK_CSBEND = 6, TRK_RFCA = 7, TRK_WAKE = 8, TRK_RADKICK = 9, TRK_MARKER = 10,
  TRK_TRWAKE = 11, TRK_MAP3 = 12
};
enum trk_aperture { TRK_APER_NONE = 0, TRK_APER_RECT = 1, TRK_APER_ELLIPSE = 2 };
enum trk_wake_mode { TRK_WAKE_FP64 = 0, TRK_WAKE_FP32_MFMA = 1 };

typedef struct trk_element {
  int32_t kind;      /* enum trk_kind */
  int32_t aperture;  /* enum trk_aperture */
  int32_t order;     /* TRK_MULT order, 1..8; TRK_QUAD 0..2 second order, 3 third */
  int32_t nsteps;    /* TRK_KQUAD/TRK_CSBEND integration steps, >= 1 */
  int32_t nbins;     /* TRK_WAKE bins, 2..TRK_MAX_BINS; TRK_TRWAKE 2..TRK_MAX_TRBINS */
  int32_t reserved;
  double L, k, angle;
  double volt, phase, freq;
  double wake_A, wake_tau0, wake_omega, charge;
  double sigma;
  double ax, ay;
  const double *coef; /* TRK_MAP2: 168, TRK_MAP3: 504 host doubles, copied at creation */
} trk_element;

#define TRK_MAX_BINS 4096
#define TRK_MAX_TRBINS 2048 /* bins of a TRK_TRWAKE */
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
  int32_t run_nt;               /* memory-bound runs: 1 non-temporal coordinate
                                   loads and stores, -1 cached, 0 automatic
                                   (non-temporal when the coordinates the run
                                   touches exceed 256 MB) */
  int32_t run_hist;             /* 0 automatic: a run that changes neither s nor
                                   the alive set (RF and wake kicks, markers, no
                                   apertures) bins the histogram of a following
                                   TRK_WAKE itself; -1 never; the results are
                                   the same */
  double p_ref_eV;              /* reference momentum at the entry of the first
                                   pass [eV/c]; raised by V cos(phase) per RFCA */
  double *moments;              /* NULL or device [passes][28]: per pass, after its
                                   last element: n, mean[6], central second
                                   moments upper triangle row-major [21]
                                   (all 0 when nobody is alive) */
} trk_opts;

/* Device workspace needed by trk_track and the collective calls for a beam of
 * n_total particles on this lattice (lat may be NULL for the standalone
 * collective calls).  The caller allocates it; contents need no
 * initialisation and are clobbered by every call. */
size_t trk_workspace_size(const trk_lattice *lat, int64_t n_total);

/* track(beam, lattice, passes): `passes` passes through the lattice.  Runs of
 * consecutive elements are fused into one kernel (coordinates loaded once,
 * kept in registers, stored once); TRK_WAKE and TRK_TRWAKE split runs.  Results do not
 * depend on the fusion depth.  Returns after enqueuing; the beam is
 * reordered (alive set first) when the last kernel completes.  With no
 * passes, no elements or n_total = 0 nothing is enqueued and opts.moments
 * is left as it was.  The call enqueues kernels only (no copies, fills or
 * allocations, and its launch sequence depends on the lattice and options,
 * not on device data), so it may be captured into a HIP graph; a replay
 * repeats the captured call on the same buffers. */
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

/* dipole histogram (the histogram of Sec. 2.2 weighted by the transverse
 * offsets): range_dev and counts_dev as trk_histogram; dipole_dev[2][nbins]
 * (int64) = per bin, the sums over its alive particles of x (row 0) and y
 * (row 1) in units of 2^-40 m, each coordinate first clamped to [-1, 1] m
 * and rounded to the nearest unit (ties to even; NaN counts 0), the sums
 * taken modulo 2^64 -- exact and independent of the summation order while
 * a bin's true sum stays below 2^23 m.  2 <= nbins <= TRK_MAX_TRBINS. */
int trk_dipole_histogram(const trk_beam *beam, int32_t nbins, double *range_dev,
                         uint32_t *counts_dev, int64_t *dipole_dev, void *workspace,
                         size_t workspace_bytes, void *stream);

/* transverse wake convolution: v_dev[2][nbins] = per plane, V[i] =
 * sum_{j<=i} D_j Wt[i-j] with D_j = dipole[j] 2^-40 (binary64),
 * Wt[m] = exp(-t/tau0) sin(omega t), t = m (smax - smin)/(nbins c)
 * (Wt[0] = 0).  TRK_WAKE_FP64: one fma chain per output, j ascending
 * (bit-exact); TRK_WAKE_FP32_MFMA: D and Wt rounded once to binary32,
 * products on FP32 matrix cores. */
int trk_trwake_convolve(const int64_t *dipole_dev, int32_t nbins, const double *range_dev,
                        double tau0, double omega, int32_t mode, double *v_dev, void *stream);

/* transverse wake kick: the convolution above, then on alive particles the
 * canonical momenta px = (1+delta) x'/sqrt(1+x'^2+y'^2) (and py) gain
 * kfac V_x(s) and kfac V_y(s), kfac = ((charge/N0) A)/p_ref_eV, V
 * interpolated as in trk_wake_kick; slopes are recomputed from the
 * momenta.  Only x' and y' change. */
int trk_trwake_kick(trk_beam *beam, const int64_t *dipole_dev, int32_t nbins,
                    const double *range_dev, const trk_wake *w, double p_ref_eV, int32_t mode,
                    void *workspace, size_t workspace_bytes, void *stream);

/* moments (Sec. 2.4 reductions): out_dev[28] = n, mean[6], central second
 * moments [21] (population normalisation) over alive particles, two passes,
 * fixed-order binary64 trees (deterministic for a given n_total); all 28
 * entries 0 when nobody is alive. */
int trk_moments(const trk_beam *beam, double *out_dev, void *workspace, size_t workspace_bytes,
                void *stream);

/* moments with compensated sums (the optional Kahan reductions of
 * Sec. 2.4): as trk_moments, but every sum is carried as a pair (s, c):
 * each thread adds its particles by Neumaier's variant of Kahan summation,
 * pairs are combined by TwoSum (the exact rounding error of each addition
 * kept), the value is s + c.  The means come from the first pass, the
 * central moments from sums of (z - mean) products.  Deterministic for a
 * given n_total; means within two units in the last place of exactly
 * rounded sums.  Same workspace as trk_moments. */
int trk_moments_compensated(const trk_beam *beam, double *out_dev, void *workspace,
                            size_t workspace_bytes, void *stream);

/* moments without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same kernels, grid and summation order as
 * trk_moments (bit-identical results), with the partial sums in a static
 * 256 KiB scratch array of the library (one copy per GPU, held until the
 * process ends; its device address is looked up on the first call made with
 * that device current).  Any n_total: the reduction's grid is capped at 1024
 * blocks, so the scratch never grows; a request that would need more is
 * refused with TRK_ERANGE.  Nothing is allocated, freed or cleared by the
 * host.  Every call on one GPU shares that GPU's scratch: calls that may
 * overlap on one GPU (other streams, other threads) race and must be
 * serialised by the caller; calls in one stream are ordered and safe. */
int trk_moments_noalloc(const trk_beam *beam, double *out_dev, void *stream);

/* compact_lost (Sec. 2.5): particles in [0, *n_alive) with lost_at >= 0 move
 * behind the survivors, ordered by lost_at descending, ties in their previous
 * order; survivors keep their order; *n_alive is decreased.  Particles at
 * and beyond the old *n_alive are not touched.  Done on the device
 * (scan, single-workgroup stable radix sort of the lost subset by a dense
 * rank of (pass, element), scatter), so the host never waits. */
int trk_compact_lost(trk_beam *beam, void *workspace, size_t workspace_bytes, void *stream);

/* The paper's two loss reorderings (Sec. 2.5), for comparison with the
 * stable one above; both act on [0, *n_alive) like it and decrease *n_alive.
 *   TRK_COMPACT_STABLE  trk_compact_lost.
 *   TRK_COMPACT_SWAP    the sparse algorithm: the k-th lost particle of the
 *                       head [0, n_new) swaps with the k-th survivor of the
 *                       tail [n_new, n_old) (index order); nothing else
 *                       moves.  Survivors do not keep their order.
 *   TRK_COMPACT_SORT    sort by key: a device radix sort of key = i
 *                       (survivor) or i + N (lost); survivors, then the lost
 *                       particles, each in their previous order.
 * n_total must be below 2^31.  The result of each mode is deterministic. */
enum trk_compact_mode { TRK_COMPACT_STABLE = 0, TRK_COMPACT_SWAP = 1, TRK_COMPACT_SORT = 2 };
int trk_compact_lost_mode(trk_beam *beam, int32_t mode, void *workspace, size_t workspace_bytes,
                          void *stream);

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
 * moments_dev: NULL or [nvar][passes][28] (as trk_opts.moments: one-pass
 * sums of the coordinates shifted by each variant's mean at the entry of the
 * call, fixed-order reductions; all 28 entries 0 for a variant with nobody
 * alive). */
int trk_track_batched(trk_batch *b, const trk_beam *beam, int32_t passes, int32_t first_pass,
                      const trk_batch_tuning *tune, double *moments_dev, void *workspace,
                      size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------ surrogate
 * Learned surrogate of a fixed lattice section (an extension beyond the
 * paper, which tracks element by element throughout; the linear part is the
 * paper's first-order transfer matrix, Sec. 3 "matrix" elements):
 *
 *   y = C + R z + D * o(N(z)),
 *
 * C = map(0) and R = Jacobian of the section map at the origin (central
 * differences of the tracker), N(z)_k = z_k / sw_k (sw = the sampler's box,
 * trk_surrogate_info.sample_half_width, which holds every admitted point, so
 * admitted inputs fill [-1, 1]; s is not an input), D_k = RMS of the residual y - (C + R z) over the training pairs
 * (D = 0 for delta, which the section leaves unchanged), and o the residual
 * network 6 -> 256 -> 256 -> 256 -> 6: h1 = silu(W1 u + b1),
 * h2 = h1 + silu(W2 h1 + b2), h3 = h2 + silu(W3 h2 + b3), o = W4 h3 + b4,
 * silu(a) = a / (1 + exp(-a)).  Matrix products run on bfloat16 matrix cores
 * with FP32 accumulation: weights rounded to bfloat16 (nearest even) from an
 * FP32 master copy, activations entered as one bfloat16 (TRK_MLP_BF16) or as
 * the sum of two (TRK_MLP_BF16X2, 16 significant bits).
 *
 * Parameter vector (FP32, TRK_MLP_NPARAM): W1[256][6], b1[256], W2[256][256],
 * b2[256], W3[256][256], b3[256], W4[6][256], b4[6]; W[out][in]. */
#define TRK_MLP_IN 6
#define TRK_MLP_HID 256
#define TRK_MLP_OUT 6
#define TRK_MLP_NPARAM 134918
enum trk_mlp_precision { TRK_MLP_BF16 = 0, TRK_MLP_BF16X2 = 1 };

typedef struct trk_mlp trk_mlp;
/* copies params_host[TRK_MLP_NPARAM]; Adam moments zero, step count 0.  The
 * handle keeps the Adam step count on the host: calls that update it
 * (trk_mlp_adam_step, trk_mlp_train) must not run from two threads at once. */
int trk_mlp_create(const float *params_host, trk_mlp **out);
void trk_mlp_destroy(trk_mlp *m);
/* copies the master parameters to the host (synchronises the stream) */
int trk_mlp_get_params(const trk_mlp *m, float *params_host, void *stream);

/* o = network(u) for n rows: u_dev[n][8] FP32 (columns 0..5, column 4 = s is
 * ignored), out_dev[n][8] FP32 (columns 0..5; 6, 7 written as 0). */
int trk_mlp_forward(const trk_mlp *m, const float *u_dev, int64_t n, float *out_dev,
                    int32_t precision, void *stream);

/* workspace of the training calls for batches of up to `batch` rows */
size_t trk_mlp_workspace_size(int32_t batch);

/* Gradient of L = (1/(6n)) sum_rows sum_k (o_k - t_k)^2 over the n rows of
 * u_dev[n][8] with targets t_dev[n][8] (FP32; columns 0..5), n a multiple of
 * 64: forward in `precision` (values saved for the backward pass), backward
 * with bfloat16 operands and FP32 accumulation, weight gradients as split-K
 * partials summed in a fixed order.  grad_dev[TRK_MLP_NPARAM] FP32 (layout
 * of the parameter vector); loss_dev: NULL or one float receiving L. */
int trk_mlp_backward(const trk_mlp *m, const float *u_dev, const float *t_dev, int32_t n,
                     int32_t precision, float *grad_dev, float *loss_dev, void *workspace,
                     size_t workspace_bytes, void *stream);

/* One Adam step (Kingma & Ba 2015) with beta1 = 0.9, beta2 = 0.999,
 * eps = 1e-8 on the master parameters, from grad_dev[TRK_MLP_NPARAM]:
 * m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
 * w <- w - lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps), evaluated in binary64
 * on binary32 state; t is the handle's step count, incremented first. */
int trk_mlp_adam_step(trk_mlp *m, const float *grad_dev, double lr, void *stream);

/* Training: epochs over n_pairs pairs u_dev[n][8], r_dev[n][8] (FP32) with
 * targets t_k = r_k inv_scale[k]; each epoch visits the pairs in the order
 * (a i + c) mod n_pairs (a, c drawn from `seed`, a coprime with n_pairs) in
 * batches of `batch` rows (the remainder is dropped), one Adam step per
 * batch, learning rate lr_min + (lr0 - lr_min)(1 + cos(pi step/steps))/2.
 * loss_dev: NULL or [epochs] floats, the sum over the epoch's batches of the
 * batch loss, divided by the number of batches. */
typedef struct trk_train_opts {
  int32_t batch;      /* rows per step, a multiple of 64 */
  int32_t epochs;
  int32_t precision;  /* forward precision while training */
  int32_t reserved;
  double lr0, lr_min;
  uint64_t seed;
} trk_train_opts;
int trk_mlp_train(trk_mlp *m, const float *u_dev, const float *r_dev, int64_t n_pairs,
                  const double inv_scale[6], const trk_train_opts *opts, float *loss_dev,
                  void *workspace, size_t workspace_bytes, void *stream);

/* A surrogate handle for a section lattice (no TRK_RFCA, TRK_WAKE, TRK_RADKICK
 * or TRK_MAP2 elements; the lattice must outlive the handle).  Creation
 * tracks 13 probes (the origin and +-h_rel hw_k along each coordinate)
 * through the section and through each of its element prefixes with the
 * tracker (synchronising `stream`) and computes on the host:
 *   C, R (central differences), the periodic Courant--Snyder parameters of
 *   the x and y blocks of R, the periodic dispersion, and the largest beta_x,
 *   beta_y, |eta| over the section's element exits (prefix maps).
 * Gate: a particle is admitted iff |z_k| <= hw_k for k != s and
 *   (xhat/a)^2 + (yhat/b)^2 <= (1 - margin)^2, xhat = sqrt(J_x betahat_x) +
 *   etahat |delta|, yhat = sqrt(J_y betahat_y), J the linear invariants of
 *   the betatron parts (each operation a separate binary64 rounding). */
typedef struct trk_surrogate_opts {
  double half_width[6];  /* training box half widths (centred at 0) */
  double margin;         /* gate margin in [0, 1) */
  double h_rel;          /* central-difference step / half width (0: 1e-4) */
  double aper_a, aper_b; /* semi-axes of the section's elliptical aperture [m] */
} trk_surrogate_opts;
typedef struct trk_surrogate_info {
  double C[6], R[36], D[6];
  double alpha_x, beta_x, gamma_x, eta, etap, alpha_y, beta_y, gamma_y;
  double beta_hat_x, beta_hat_y, eta_hat, lim;
  double sample_half_width[6]; /* box of the sampler (contains the admitted set) */
} trk_surrogate_info;
typedef struct trk_surrogate trk_surrogate;
int trk_surrogate_create(const trk_lattice *section, const trk_surrogate_opts *opts, void *stream,
                         trk_surrogate **out);
void trk_surrogate_destroy(trk_surrogate *s);
int trk_surrogate_get_info(const trk_surrogate *s, trk_surrogate_info *out);

/* workspace of the calls below for beams of up to n_total particles */
size_t trk_surrogate_workspace_size(const trk_surrogate *s, int64_t n_total);

/* admit_dev[i] = 1 if particle i < *n_alive is admitted, else 0 */
int trk_surrogate_gate(const trk_surrogate *s, const trk_beam *beam, uint8_t *admit_dev,
                       void *stream);

/* Fills beam (n_total slots; ids 0.., lost_at -1, *n_alive = n_total) with
 * admitted points drawn uniformly: candidate c = first, first+1, ... takes
 * two Philox4x32-10 blocks with counters (c_lo, c_hi, 5, 0) and
 * (c_lo, c_hi, 5, 1), key = seed; z_k = (2 u_k - 1) w_k with
 * u_k = (word_k + 1/2) 2^-32, w = sample_half_width; admitted candidates are
 * kept in candidate order.  *next_out (host) = first candidate not examined.
 * Synchronises the stream once per round of candidates. */
int trk_surrogate_sample(const trk_surrogate *s, uint64_t seed, uint64_t first, trk_beam *beam,
                         uint64_t *next_out, void *workspace, size_t workspace_bytes,
                         void *stream);

/* Training pairs: the admitted particles of `beam` (in their order) are
 * tracked through the section; survivors j = 0 .. *n_pairs_dev - 1 give
 * u_dev[j][8] = N(z_in) (FP32) and r_dev[j][8] = y - (C + R z_in) (FP32,
 * columns 0..4).  The beam itself is not modified. */
int trk_surrogate_pairs(const trk_surrogate *s, const trk_beam *beam, float *u_dev, float *r_dev,
                        int64_t *n_pairs_dev, void *workspace, size_t workspace_bytes,
                        void *stream);

/* D_k = sqrt(mean over the n rows of r_k^2) for k = 0..4 (synchronises) */
int trk_surrogate_fit_scale(trk_surrogate *s, const float *r_dev, int64_t n, void *workspace,
                            size_t workspace_bytes, void *stream);

/* One pass through the section for the alive particles of `beam`: admitted
 * ones get the surrogate output (in place), the others are tracked element
 * by element (pass index first_pass in their loss records); the beam is
 * then compacted as trk_track leaves it.  n_admitted_dev: NULL or the
 * number of admitted particles. */
int trk_surrogate_apply(const trk_surrogate *s, const trk_mlp *m, trk_beam *beam,
                        int32_t first_pass, int32_t precision, int64_t *n_admitted_dev,
                        void *workspace, size_t workspace_bytes, void *stream);

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

/* Machine ceilings on the box, for the rooflines.  trk_probe_stream: mode 0
 * copies src to dst (dst[i] = src[i] + 1; n doubles read and n written),
 * mode 1 only reads src (dst[b] = the sum of workgroup b's elements, so dst
 * holds `blocks` doubles), mode 2 copies as mode 0 with non-temporal loads
 * and stores; 256-thread workgroups, grid-stride, four loads in
 * flight per lane.  trk_probe_fma: `blocks` x 256 lanes each run 8
 * independent chains of `iters` binary64 fmas (2 flops each) and store one
 * value, out_dev[blocks * 256].  Both enqueue one kernel; EINVAL for a bad
 * mode, n < 0, iters < 0 or blocks outside 1..2^20, EPTR for host pointers. */
int trk_probe_stream(const double *src_dev, double *dst_dev, int64_t n, int32_t mode,
                     int32_t blocks, void *stream);
int trk_probe_fma(double *out_dev, int32_t iters, int32_t blocks, void *stream);

/* ------------------------------------------------------------------ misc */
const char *trk_status_string(int status);
const char *trk_last_error(void);
/* per-kernel-class device time (ms) and launch count accumulated while
 * enabled, from start and stop events that each timed kernel's own dispatch
 * records (hipExtLaunchKernel: no event packet between kernels); class 0 =
 * fused element run, class 1 = surrogate network inference, class 2 = wake
 * histogram, class 3 = wake convolution (inside trk_track).  trk_profile_enable: `on` is a bit mask of the classes
 * to time (bit c = class c; 0 stops timing); a nonzero mask also clears the
 * accumulated figures. */
int trk_profile_enable(int32_t on);
int trk_profile_read(int32_t kernel_class, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif
