// run.hip -- the fused element-run kernel.
//
// One lane owns one particle: its six coordinates are loaded once from the
// structure-of-arrays beam (coalesced 8-byte loads), a run of consecutive
// elements -- possibly several whole passes -- is applied in registers and
// the coordinates are stored once.  This is the register-resident form of
// the paper's particle accessor (Sec. 2.1: at most one read and one write per
// coordinate per kernel), extended from one element to a run of elements.
//
// Element records are read at wave-uniform addresses, so the compiler keeps
// them in scalar registers and the element switch is a scalar branch.  A lane
// whose particle fails an aperture stops updating (its coordinates freeze at
// that element's exit) and records (pass << 32) | element.
//
// Optional fused reductions: per-pass moment partials (shifted sums of the
// survivors, one row of 28 per block) and the (min, max) of s over survivors
// at the end of the run, which feeds the histogram of a following wake.
#include <cfloat>

#include <utility>

#include "apply.h"
#include "reduce.h"

namespace trk {

// s/delta-only runs (RF cavities, wake kicks, longitudinal maps), software
// pipelined: the (s, delta) of a thread's next kP particles are loaded before
// the current kP go through the elements, so each wave keeps its next loads
// in flight while it computes.  The element switch sits outside the particle
// loop, so the wake-table reads of all kP particles are issued together.
template <uint32_t kFeat, int kP, bool kNT>
__device__ __forceinline__ void run_long(const RunArgs &a) {
  const ConstElems elems = (ConstElems)a.elems;
  const ConstPool pool = (ConstPool)a.pool;
  const ElemCtx cx{a.vc, a.nv, a.v0, a.wake_v, a.wake_par, a.seed_lo, a.seed_hi};
  const int64_t n = min(*a.n_alive, a.n_total);
  if (a.zero_buf != nullptr && blockIdx.x == 0)
    for (int i = threadIdx.x; i < a.zero_n; i += kBlock) a.zero_buf[i] = 0u;

  double smin = __builtin_huge_val(), smax = -__builtin_huge_val();
  const int64_t nthr = static_cast<int64_t>(gridDim.x) * kBlock;
  const int64_t first = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t step = nthr * kP;
  const int64_t ntot = a.n_total;
  double *const zs = a.z[4];
  double *const zd = a.z[5];
  // the next wake's histogram, binned here when the run changes neither s
  // nor the alive set (its range is the last histogram's, exact)
  extern __shared__ uint32_t hsub[];
  const bool hist = a.hist_out != nullptr;
  double hmn = 0.0, hinv = 0.0;
  if (hist) {
    for (int j = threadIdx.x; j < a.hist_nbins; j += kBlock) hsub[j] = 0u;
    hmn = a.hist_range[0];
    const double width = a.hist_range[1] - hmn;
    hinv = width > 0.0 ? static_cast<double>(a.hist_nbins) / width : 0.0;
    __syncthreads();
  }
  double ns[kP], nd[kP];
  // the first loads are bounded by the array length, so they need not wait
  // for the device-side particle count; later ones by the count
#pragma unroll
  for (int q = 0; q < kP; ++q) {
    const int64_t i = first + q * nthr;
    const bool inb = i < ntot;
    if constexpr (kNT) {
      ns[q] = inb ? __builtin_nontemporal_load(zs + i) : 0.0;
      nd[q] = inb ? __builtin_nontemporal_load(zd + i) : 0.0;
    } else {
      ns[q] = inb ? zs[i] : 0.0;
      nd[q] = inb ? zd[i] : 0.0;
    }
  }
  for (int64_t base = first; base < n; base += step) {
    double sv[kP], dv[kP];
    bool act[kP];
#pragma unroll
    for (int q = 0; q < kP; ++q) {
      sv[q] = ns[q];
      dv[q] = nd[q];
      act[q] = base + q * nthr < n;
    }
    const int64_t nb = base + step;
#pragma unroll
    for (int q = 0; q < kP; ++q) {
      const int64_t i = nb + q * nthr;
      const bool inb = i < n;
      if constexpr (kNT) {
        ns[q] = inb ? __builtin_nontemporal_load(zs + i) : 0.0;
        nd[q] = inb ? __builtin_nontemporal_load(zd + i) : 0.0;
      } else {
        ns[q] = inb ? zs[i] : 0.0;
        nd[q] = inb ? zd[i] : 0.0;
      }
    }
    for (int p = 0; p < a.npass; ++p)
      for (int e = a.e0; e < a.e1; ++e) apply_long_q<kFeat, kP>(elems[e], pool, cx, p, sv, dv, act);
#pragma unroll
    for (int q = 0; q < kP; ++q) {
      if (!act[q]) continue;
      const int64_t i = base + q * nthr;
      if ((a.stmask >> 4) & 1u) {
        if constexpr (kNT)
          __builtin_nontemporal_store(sv[q], zs + i);
        else
          zs[i] = sv[q];
      }
      if ((a.stmask >> 5) & 1u) {
        if constexpr (kNT)
          __builtin_nontemporal_store(dv[q], zd + i);
        else
          zd[i] = dv[q];
      }
      smin = fmin(smin, sv[q]);
      smax = fmax(smax, sv[q]);
      if (hist) {
        const double f = (sv[q] - hmn) * hinv;
        if (f >= 0.0) atomicAdd(hsub + min(static_cast<int>(f), a.hist_nbins - 1), 1u);
      }
    }
  }
  if (hist) {
    __syncthreads();
    uint32_t *out = a.hist_out + (blockIdx.x % kHistCopies) * a.hist_nbins;
    for (int j = threadIdx.x; j < a.hist_nbins; j += kBlock) {
      const uint32_t c = hsub[j];
      if (c != 0u) atomicAdd(out + j, c);
    }
  }
  if (a.mm_part != nullptr) {
    block_minmax(smin, smax);
    if (threadIdx.x == 0) {
      a.mm_part[2 * blockIdx.x] = smin;
      a.mm_part[2 * blockIdx.x + 1] = smax;
    }
  }
}

// kP particles per thread, strided by the grid size so every load and store
// stays coalesced; the kP particles go through each element together, so an
// element record is read once per kP particles and the loads of all kP are
// in flight at once.  Loads are issued for indices below the array length
// before the device-side particle count arrives (they stay in bounds), so
// the count's latency is not paid twice.  kLong: the run reads and writes
// only s and delta, handled by run_long.  The moments variant makes one pass
// over the grid with kP particles per thread, so that every thread reaches
// the per-pass block reductions.  kNT: the coordinates are streamed with
// non-temporal loads and stores.
template <uint32_t kFeat, bool kMom, int kP, bool kLong, bool kNT = false>
__global__ __launch_bounds__(kBlock) void k_run(const RunArgs a) {
  if constexpr (kLong) {
    run_long<kFeat, kP, kNT>(a);
    return;
  }
  const ConstElems elems = (ConstElems)a.elems;
  const ConstPool pool = (ConstPool)a.pool;
  const ElemCtx cx{a.vc, a.nv, a.v0, a.wake_v, a.wake_par, a.seed_lo, a.seed_hi};
  const int64_t n = min(*a.n_alive, a.n_total);
  if (a.zero_buf != nullptr && blockIdx.x == 0)
    for (int i = threadIdx.x; i < a.zero_n; i += kBlock) a.zero_buf[i] = 0u;

  double smin = __builtin_huge_val(), smax = -__builtin_huge_val();
  const int64_t nthr = static_cast<int64_t>(gridDim.x) * kBlock;
  const int64_t first = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t step = kMom ? 0 : nthr * kP;
  const int64_t ntot = a.n_total;
  // the next wake's histogram, binned here when the run changes neither s
  // nor the alive set (its range is the last histogram's, exact)
  extern __shared__ uint32_t hsub[];
  const bool hist = !kMom && a.hist_out != nullptr;
  double hmn = 0.0, hinv = 0.0;
  if (hist) {
    for (int j = threadIdx.x; j < a.hist_nbins; j += kBlock) hsub[j] = 0u;
    hmn = a.hist_range[0];
    const double width = a.hist_range[1] - hmn;
    hinv = width > 0.0 ? static_cast<double>(a.hist_nbins) / width : 0.0;
    __syncthreads();
  }

  for (int64_t it = 0, base = first; kMom ? (it < 1) : (base < ntot); ++it, base += step) {
    double z[kP][6];
    bool act[kP], alive[kP];
    int64_t rec[kP];
    uint32_t pid[kP];
#pragma unroll
    for (int q = 0; q < kP; ++q) {
      const int64_t i = base + q * nthr;
      const bool inb = i < ntot;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const bool want = ((a.ldmask >> k) & 1u) != 0;
        if constexpr (kNT)
          z[q][k] = (inb && want) ? __builtin_nontemporal_load(a.z[k] + i) : 0.0;
        else
          z[q][k] = (inb && want) ? a.z[k][i] : 0.0;
      }
      pid[q] = (inb && ((a.ldmask >> 6) & 1u)) ? a.id[i] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kP; ++q) {
      act[q] = base + q * nthr < n;
      // A particle lost earlier in the same call still holds its slot.  The
      // 64 slots of a wave share one loss flag (a wave-uniform load); only
      // flagged groups read the loss records.
      if (a.chk_lost) {
        int64_t g = __builtin_amdgcn_readfirstlane(static_cast<int>((base + q * nthr) >> 6));
        const int64_t glast = ntot > 0 ? (ntot - 1) >> 6 : 0;
        g = g < 0 ? 0 : (g < glast ? g : glast);  // in bounds even with no lane active
        if (act[q] && a.lost_flag[g] != 0u) act[q] = a.lost_at[base + q * nthr] < 0;
      }
      alive[q] = act[q];
      rec[q] = -1;
    }
    for (int p = 0; p < a.npass; ++p) {
      const uint32_t gp = static_cast<uint32_t>(a.pass0 + p);
      for (int e = a.e0; e < a.e1; ++e) {
        const DevElem E = elems[e];
#pragma unroll
        for (int q = 0; q < kP; ++q)
          apply<kFeat>(E, pool, cx, p, gp, e, z[q], alive[q], rec[q], pid[q]);
      }
      if constexpr (kMom) {
        double *row = a.mom_part + (static_cast<int64_t>(p) * gridDim.x + blockIdx.x) * 28;
        if constexpr (kP == 1) {
          double d[6];
#pragma unroll
          for (int k = 0; k < 6; ++k) d[k] = alive[0] ? z[0][k] - a.mom_shift[k] : 0.0;
          block_moment_row(alive[0] ? 1.0 : 0.0, d, row);
        } else {
          double d[kP][6];
#pragma unroll
          for (int q = 0; q < kP; ++q)
#pragma unroll
            for (int k = 0; k < 6; ++k) d[q][k] = alive[q] ? z[q][k] - a.mom_shift[k] : 0.0;
          block_moment_row_multi<kP>(alive, d, row);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kP; ++q) {
      if (!act[q]) continue;
      const int64_t i = base + q * nthr;
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if ((a.stmask >> k) & 1u) {
          if constexpr (kNT)
            __builtin_nontemporal_store(z[q][k], a.z[k] + i);
          else
            a.z[k][i] = z[q][k];
        }
      if (rec[q] >= 0) {
        a.lost_at[i] = rec[q];
        a.lost_flag[i >> 6] = 1u;
      }
      if (alive[q]) {
        smin = fmin(smin, z[q][4]);
        smax = fmax(smax, z[q][4]);
        if (hist) {
          const double f = (z[q][4] - hmn) * hinv;
          if (f >= 0.0) atomicAdd(hsub + min(static_cast<int>(f), a.hist_nbins - 1), 1u);
        }
      }
    }
    if constexpr (!kMom) {
      if (base + nthr * kP >= n) break;  // nothing alive further on
    }
  }
  if (hist) {
    __syncthreads();
    uint32_t *out = a.hist_out + (blockIdx.x % kHistCopies) * a.hist_nbins;
    for (int j = threadIdx.x; j < a.hist_nbins; j += kBlock) {
      const uint32_t c = hsub[j];
      if (c != 0u) atomicAdd(out + j, c);
    }
  }
  if (a.mm_part != nullptr) {
    block_minmax(smin, smax);
    if (threadIdx.x == 0) {
      a.mm_part[2 * blockIdx.x] = smin;
      a.mm_part[2 * blockIdx.x + 1] = smax;
    }
  }
}

// light element families (no kick-drift, random or generic-map elements)
// are memory bound: several particles per thread
constexpr bool light(uint32_t f) { return (f & (F_KD | F_RNG | F_GEN)) == 0; }
constexpr bool longit_ok(uint32_t f) { return (f & ~(F_RF | F_WAKE)) == 0; }

template <uint32_t kFeat, bool kLong, bool kNT>
void launch_ppt_nt(const RunArgs &a, int grid, hipStream_t st) {
  // a run-binned histogram keeps its counts in LDS
  const size_t lds = a.hist_out != nullptr ? sizeof(uint32_t) * a.hist_nbins : 0;
  switch (a.ppt) {
    case 8: TRK_LAUNCH((k_run<kFeat, false, 8, kLong, kNT>), dim3(grid), dim3(kBlock), lds, st, a); break;
    case 4: TRK_LAUNCH((k_run<kFeat, false, 4, kLong, kNT>), dim3(grid), dim3(kBlock), lds, st, a); break;
    case 2: TRK_LAUNCH((k_run<kFeat, false, 2, kLong, kNT>), dim3(grid), dim3(kBlock), lds, st, a); break;
    default: TRK_LAUNCH((k_run<kFeat, false, 1, kLong, kNT>), dim3(grid), dim3(kBlock), lds, st, a); break;
  }
}

template <uint32_t kFeat, bool kLong>
void launch_ppt(const RunArgs &a, int grid, hipStream_t st) {
  if (a.nt)
    launch_ppt_nt<kFeat, kLong, true>(a, grid, st);
  else
    launch_ppt_nt<kFeat, kLong, false>(a, grid, st);
}

template <uint32_t kFeat>
void launch_feat(const RunArgs &a, int grid, hipStream_t st) {
  if (a.mom) {
    if (a.ppt >= 2)
      TRK_LAUNCH((k_run<kFeat, true, 2, false>), dim3(grid), dim3(kBlock), 0, st, a);
    else
      TRK_LAUNCH((k_run<kFeat, true, 1, false>), dim3(grid), dim3(kBlock), 0, st, a);
  } else if constexpr (light(kFeat)) {
    if constexpr (longit_ok(kFeat)) {
      if (a.longit) {
        launch_ppt<kFeat, true>(a, grid, st);
        return;
      }
    }
    launch_ppt<kFeat, false>(a, grid, st);
  } else {
    // heavy runs: one or two particles per thread
    const size_t lds = a.hist_out != nullptr ? sizeof(uint32_t) * a.hist_nbins : 0;
    if (a.ppt >= 2)
      TRK_LAUNCH((k_run<kFeat, false, 2, false>), dim3(grid), dim3(kBlock), lds, st, a);
    else
      TRK_LAUNCH((k_run<kFeat, false, 1, false>), dim3(grid), dim3(kBlock), lds, st, a);
  }
}

int run_shape(RunArgs &a, int64_t n_total, int ppt_req, int cap_req) {
  if (a.mom) {
    // every thread reaches the per-pass block reductions: no grid stride
    a.ppt = ppt_req >= 2 ? 2 : 1;
    const int64_t g = (n_total + static_cast<int64_t>(kBlock) * a.ppt - 1) / (kBlock * a.ppt);
    return static_cast<int>(g < 1 ? 1 : g);
  }
  // light runs with RF cavities or wakes on all six coordinates carry the
  // registers of sines, square roots and divisions: one particle per thread
  const bool rfw = !a.longit && (a.feat & (F_RF | F_WAKE)) != 0;
  int ppt = ppt_req > 0 ? ppt_req
                        : (a.longit ? kLongPPT : (light(a.feat) && !rfw ? kLightPPT : 1));
  if (!light(a.feat)) ppt = ppt >= 2 ? 2 : 1;
  ppt = ppt >= 8 ? 8 : (ppt >= 4 ? 4 : (ppt >= 2 ? 2 : 1));
  a.ppt = ppt;
  const int64_t want = (n_total + static_cast<int64_t>(kBlock) * ppt - 1) / (kBlock * ppt);
  // streaming light runs cover the array in one sweep of the grid; the others stride
  const int64_t cap =
      cap_req > 0 ? cap_req
                  : (a.longit ? kLongRunGrid : (light(a.feat) && !rfw ? want : kMaxRunGrid));
  return static_cast<int>(want < 1 ? 1 : (want > cap ? cap : want));
}

template <uint32_t... kF>
void dispatch(uint32_t feat, const RunArgs &a, int grid, hipStream_t st,
              std::integer_sequence<uint32_t, kF...>) {
  ((feat == kF ? (launch_feat<kF>(a, grid, st), 0) : 0), ...);
}

hipError_t launch_run(const RunArgs &a, int grid, hipStream_t st) {
  dispatch(a.feat & F_ALL, a, grid, st, std::make_integer_sequence<uint32_t, F_ALL + 1>{});
  return hipGetLastError();
}

}  // namespace trk
