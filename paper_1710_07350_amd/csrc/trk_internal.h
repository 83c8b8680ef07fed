// trk_internal.h -- device records, kernel arguments and launch helpers
// shared by the HIP translation units of libtrk.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/trk.h"

namespace trk {

// Start and stop events for the next kernel this thread launches through
// TRK_LAUNCH (set by the profiling wrapper, consumed by that one launch).
// The extended launch has the dispatch packet itself record the kernel's
// start and end, so no event packet sits between two kernels of the stream.
struct KernelEvents {
  hipEvent_t start, stop;
};
extern thread_local KernelEvents g_kernel_events;

#define TRK_LAUNCH(kernel, grid, block, lds, st, ...)                                           \
  do {                                                                                        \
    if (::trk::g_kernel_events.start != nullptr) {                                            \
      const ::trk::KernelEvents ev_ = ::trk::g_kernel_events;                                 \
      ::trk::g_kernel_events = ::trk::KernelEvents{nullptr, nullptr};                         \
      hipExtLaunchKernelGGL(kernel, grid, block, lds, st, ev_.start, ev_.stop, 0, __VA_ARGS__); \
    } else {                                                                                  \
      hipLaunchKernelGGL(kernel, grid, block, lds, st, __VA_ARGS__);                          \
    }                                                                                         \
  } while (0)

constexpr int kBlock = 256;
// copies of the counts a run-binned histogram merges into (spreads the
// same-address contention of up to kMaxRunGrid workgroups)
constexpr int kHistCopies = 8;
constexpr int kMaxVar = 96;        // pass-varying constants per fused launch
constexpr int kMaxGridStride = 2048;
constexpr int kMaxPassesPerLaunch = 64;
constexpr int kLightPPT = 2;       // particles per thread of memory-bound runs
constexpr int kLongPPT = 4;        // ... of runs that touch only s and delta
constexpr int kLongRunGrid = 1024; // grid-stride cap of those runs (4 blocks per CU)
constexpr int kMaxRunGrid = 4096;  // grid-stride cap of the run kernel

// Device element kinds after host-side classification.  MAP2 maps are
// evaluated through one of three code paths with identical arithmetic:
// P1 = the thick-quad sparsity pattern, P2 = identity + R56 + T566, GEN = any.
enum DevKind : int32_t {
  K_EDRIFT = 1,
  K_MAP2_P1 = 2,
  K_MAP2_P2 = 3,
  K_MAP2_GEN = 4,
  K_MULT = 5,
  K_KQUAD = 6,
  K_CSBEND = 7,
  K_RFCA = 8,
  K_WAKE = 9,
  K_RADKICK = 10,
  K_MARKER = 11,
  K_TRWAKE = 12,
  K_MAP3_P3 = 13,
  K_MAP3_GEN = 14,
};

// Element families present in a run; the run kernel is instantiated per set
// so that a run of light elements does not pay the registers of heavy ones.
enum Feat : uint32_t { F_KD = 1, F_RF = 2, F_WAKE = 4, F_RNG = 8, F_GEN = 16, F_ALL = 31 };

// 80-byte record read by every lane of a wave at the same address (scalar
// loads); `off` indexes the lattice's constant pool.
struct DevElem {
  int32_t kind, aper, ip, off;  // ip: MULT order | KQUAD/CSBEND steps | WAKE bins
  int32_t vslot, pad0, pad1, pad2;
  double a0, a1;                // RECT: (X, Y); ELLIPSE: (1/a, 1/b)
  double p0, p1, p2, p3;        // kind-specific scalars
};
static_assert(sizeof(DevElem) == 80, "DevElem layout");

// Pool layouts (offsets from DevElem::off):
//   MAP2_P1   24: x:(R11 R12 T116 T126) x':(R21 R22 T216 T226)
//                 y:(R33 R34 T336 T346) y':(R43 R44 T436 T446)
//                 s:(R55 T511 T512 T522 T533 T534 T544) delta:(R66)
//   MAP2_P2    8: R11 R22 R33 R44 R55 R56 R66 T566
//   MAP2_GEN 168: C[6] R[6][6] T[6][21]
//   MAP3_P3   38: the 24 of MAP2_P1, then x:(U1166 U1266) x':(U2166 U2266)
//                 y:(U3366 U3466) y':(U4366 U4466)
//                 s:(U5116 U5126 U5226 U5336 U5346 U5446)
//   MAP3_GEN 504: C[6] R[6][6] T[6][21] U[6][56]
//   KQUAD      7: kq[4] dl[3]
//   CSBEND    23: kA[4] kB[4] cph[3] sph[3] vers[3] rs[3] dl[3]
// Scalars: EDRIFT p0 = L; MULT p0 = KnL/n!; RFCA p0 = k/2, p1 = sin(phase),
//   p2 = cos(phase), p3 = V; RADKICK p0 = sigma; WAKE, TRWAKE ip = nbins.
// Pass-varying constants vc[slot] = (a, b): RFCA (P_in, 1/P_out), WAKE and
// TRWAKE (kfac, 0).

struct RunArgs {
  double *z[6];
  uint32_t *id;
  int64_t *lost_at;
  const int64_t *n_alive;
  const DevElem *elems;
  const double *pool;
  int32_t e0, e1;       // element range of each pass
  int32_t pass0, npass; // global first pass, passes in this launch
  int32_t v0, nv;       // varying-constant slots of [e0, e1)
  uint32_t seed_lo, seed_hi;
  uint32_t ldmask, stmask;  // bit k: coordinate k loaded / stored; bit 6: id
  uint32_t feat;            // element families present (selects the instantiation)
  int32_t longit;           // run reads/writes only s and delta, no apertures
  int32_t chk_lost;         // slots below *n_alive may hold lost particles (lazy compaction)
  uint32_t *lost_flag;      // [ceil(n_total/64)]: nonzero when a particle of those 64 slots
                            // was lost since the flags were cleared (gates the lost_at read)
  int32_t ppt;              // particles per thread (1, 2, 4, 8)
  int32_t nt;               // light runs: non-temporal coordinate loads and stores
  int32_t grid_cap;         // grid-stride cap
  int64_t n_total;          // array length (bound of speculative loads)
  const double *wake_v;     // V[nbins] when elements[e0] is a WAKE; Vx, Vy for a TRWAKE
  const double *wake_par;   // (smin, 1/delta)
  double *mm_part;          // [gridDim.x][2] (min s, max s) of survivors, or null
  // Histogram of the next wake binned in this run (two-coordinate runs that
  // change neither s nor the alive set): hist_out[kHistCopies][hist_nbins]
  // (zeroed beforehand) receives the counts of the final s over
  // [hist_range[0], hist_range[1]], workgroup b adding to copy b % kHistCopies.
  uint32_t *hist_out;
  const double *hist_range;
  int32_t hist_nbins;
  uint32_t *zero_buf;       // zeroed by block 0 when non-null
  int32_t zero_n;
  int32_t mom;              // per-pass moment partials
  double *mom_part;         // [npass][gridDim.x][28]
  const double *mom_shift;  // [6]
  double vc[kMaxVar][2];
};

// Batched launch over concatenated variants (see batch.hip).
struct BatchArgs {
  double *z[6];
  uint32_t *id;
  int64_t *lost_at;
  const int64_t *seg_off;    // [nvar+1] particle offsets of the variants
  const int64_t *chunk_off;  // [nvar+1] ticket offsets (chunks of kBlock*ppt particles)
  const uint64_t *seeds;     // [nvar] random-kick keys
  const DevElem *elems;      // [nvar][nelem]
  const double *pool;
  int32_t nelem, nvar, pass0, npass;
  uint32_t ldmask, stmask;
  uint32_t *ticket;          // zeroed before the launch
  int64_t total;             // tickets
  double *mom_part;          // [total][npass][28] or null
  const double *mom_shift;   // [nvar][6] moment shift: each variant's mean at entry
  double *mean_part;         // [total][7] (n, sum z_k) per chunk, for the shift
};
hipError_t launch_batch(const BatchArgs &a, uint32_t feat, int ppt, int grid, hipStream_t st);
// the variants' means at entry into a.mom_shift (a.mean_part as scratch)
hipError_t launch_batch_mean(const BatchArgs &a, int ppt, hipStream_t st);
hipError_t launch_batch_mom_finalize(const double *part, const int64_t *chunk_off,
                                     const double *shift, int nvar, int npass, double *out,
                                     int out_pass0, int out_passes, hipStream_t st);

// ---------------------------------------------------------------- workspace
struct Workspace {
  double *mm_part;     // [kMaxGridStride][2]
  uint32_t *counts;    // [TRK_MAX_BINS + 64], then the dipole sums:
  int64_t *dip;        // [2][TRK_MAX_TRBINS] (same allocation, zeroed with the counts)
  uint32_t *lost_flag; // [ceil(n/64)] loss flags of 64-slot groups
  double *range;       // [2]
  uint32_t *hcounts[2];  // [kHistCopies][TRK_MAX_BINS] each: run-binned histograms, alternating
  double *wake_par;    // [2]
  double *wake_v;      // [2 * TRK_MAX_BINS]
  double *mom_shift;   // [6]
  double *mom_tmp;     // [28]
  double *mom_part;    // [kMaxPassesPerLaunch][nblk][28]
  int64_t *cmp_blk;    // [nblk][10]
  int64_t *cmp_hdr;    // [16]
  uint64_t *key_a, *key_b;  // [n]
  uint32_t *pos_a, *pos_b;  // [n]
  double *tz[6];       // [n] scatter staging
  uint32_t *tid;       // [n]
  int64_t *tlost;      // [n]
  uint32_t *rs_cnt;    // [256][compaction tiles] digit counts of the multi-block sort
  uint32_t *rs_tot;    // [256]
  void *sort_tmp;      // device radix-sort scratch of the sort-by-key compaction
  size_t sort_tmp_bytes;
};
size_t workspace_bytes(int64_t n_total);
Workspace carve_workspace(void *base, int64_t n_total);

inline int64_t nblocks(int64_t n) { return (n + kBlock - 1) / kBlock; }

// ---------------------------------------------------------------- launchers
// (each returns hipSuccess or the launch error; all asynchronous)
hipError_t launch_run(const RunArgs &a, int grid, hipStream_t st);
hipError_t launch_minmax(const double *s, const int64_t *n_alive, int64_t n_total, double *mm_part,
                         int grid, uint32_t *zero_buf, int zero_n, hipStream_t st);
// x, y, dip non-null: also the dipole sums dip[2][nbins] (zeroed beforehand)
hipError_t launch_histogram(const double *s, const int64_t *n_alive, int64_t n_total,
                            const double *mm_part, int mm_n, int nbins, uint32_t *counts,
                            double *range, hipStream_t st, const double *x = nullptr,
                            const double *y = nullptr, int64_t *dip = nullptr);
// transverse: v[2][nbins] from dip[2][nbins]
hipError_t launch_convolve_tr(const int64_t *dip, int nbins, const double *range, double tau0,
                              double omega, int mode, double *v, double *wake_par, hipStream_t st,
                              uint32_t *zbuf = nullptr, int zn = 0);
hipError_t launch_trwake_kick(double *const z[6], const int64_t *n_alive, int64_t n_total,
                              const double *v, const double *wake_par, int nbins, double kfac,
                              hipStream_t st);
// v: the convolution; wake_par: (smin, nbins/width) or null.  counts holds
// ncopy copies [ncopy][nbins] whose sum is the histogram; zbuf (or null):
// zn words zeroed by the first workgroup (a buffer the next run bins into)
hipError_t launch_convolve(const uint32_t *counts, int nbins, const double *range, double tau0,
                           double omega, int mode, double *v, double *wake_par, hipStream_t st,
                           int ncopy = 1, uint32_t *zbuf = nullptr, int zn = 0);
hipError_t launch_wake_kick(double *s, double *dp, const int64_t *n_alive, int64_t n_total,
                            const double *v, const double *wake_par, int nbins, double kfac,
                            hipStream_t st);
// launch shape of a run: fills a.ppt and returns the grid (a.longit, a.feat,
// a.mom set; ppt_req/cap_req 0 = automatic)
int run_shape(RunArgs &a, int64_t n_total, int ppt_req, int cap_req);
hipError_t launch_mom_partial(double *const z[6], const int64_t *n_alive, int64_t n_total,
                              const double *shift, double *part, int grid, hipStream_t st);
hipError_t launch_mom_finalize(const double *part, int nrows, int npass, const double *shift,
                               double *out, int out_stride, double *mean_out, hipStream_t st);
// compensated two-pass moments: rows of 56 (28 sums, 28 compensations)
hipError_t launch_mom_partial_c(double *const z[6], const int64_t *n_alive, int64_t n_total,
                                const double *shift, double *part, int grid, hipStream_t st);
hipError_t launch_mom_finalize_c(const double *part, int nrows, const double *shift, double *out,
                                 double *mean_out, hipStream_t st);
hipError_t launch_compact(double *const z[6], uint32_t *id, int64_t *lost_at, int64_t *n_alive,
                          int64_t n_total, const Workspace &w, hipStream_t st);
// the paper's sparse swap (TRK_COMPACT_SWAP) or sort by key (TRK_COMPACT_SORT)
hipError_t launch_compact_variant(int mode, double *const z[6], uint32_t *id, int64_t *lost_at,
                                  int64_t *n_alive, int64_t n_total, const Workspace &w,
                                  hipStream_t st);
size_t sortkey_temp_bytes(int64_t n_total);
int64_t compact_tiles(int64_t n_total);  // 4096-slot tiles of the compaction kernels
hipError_t launch_zero_u32(uint32_t *p, int n, hipStream_t st);
hipError_t launch_elementary(int fn, const double *x, const double *y, double *out, int64_t n,
                             hipStream_t st);
hipError_t launch_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out, int64_t n,
                         hipStream_t st);
hipError_t launch_gauss(const uint32_t *id, uint32_t step, uint32_t tag, uint64_t seed,
                        double *out, int64_t n, hipStream_t st);
// machine probes: streaming (mode 0 copy, 1 read-only) and FP64 FMA ceilings
hipError_t launch_probe_stream(const double *src, double *dst, int64_t n, int mode, int grid,
                               hipStream_t st);
hipError_t launch_probe_fma(double *out, int iters, int grid, hipStream_t st);

}  // namespace trk
