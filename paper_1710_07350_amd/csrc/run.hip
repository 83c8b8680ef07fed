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

#include "elements.h"
#include "reduce.h"

namespace trk {

// Rarely executed handlers stay out of line so that their registers do not
// count against the hot element loop.
__device__ __noinline__ void radkick_call(double &dp, double sigma, uint32_t pid, uint32_t gp,
                                          uint32_t klo, uint32_t khi) {
  dp = fma(sigma, dm::gauss(pid, gp, 2u, klo, khi), dp);
}
__device__ __noinline__ void map_gen_call(double (&z)[6], const double *__restrict__ c) {
  el::map_gen(z, c);
}

template <uint32_t kFeat, bool kMom>
__global__ __launch_bounds__(kBlock) void k_run(const RunArgs a) {
  const int64_t n = *a.n_alive;
  if (a.zero_buf != nullptr && blockIdx.x == 0)
    for (int i = threadIdx.x; i < a.zero_n; i += kBlock) a.zero_buf[i] = 0u;

  double smin = __builtin_huge_val(), smax = -__builtin_huge_val();
  const int64_t first = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
  const int64_t stride = kMom ? 0 : static_cast<int64_t>(gridDim.x) * kBlock;

  // moments variant: exactly one particle per thread (every thread must reach
  // the per-pass block reductions); otherwise a grid-stride loop
  for (int64_t it = 0, i = first; kMom ? (it < 1) : (i < n); ++it, i += stride) {
    const bool act = i < n;
    double z[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) z[k] = (act && ((a.ldmask >> k) & 1u)) ? a.z[k][i] : 0.0;
    const uint32_t pid = (act && ((a.ldmask >> 6) & 1u)) ? a.id[i] : 0u;
    bool alive = act;
    int64_t rec = -1;

    for (int p = 0; p < a.npass; ++p) {
      const uint32_t gp = static_cast<uint32_t>(a.pass0 + p);
      for (int e = a.e0; e < a.e1; ++e) {
        const DevElem E = a.elems[e];
        if (alive) {
          const double *__restrict__ c = a.pool + E.off;
          switch (E.kind) {
            case K_EDRIFT: el::edrift(z, E.p0); break;
            case K_MAP2_P1: el::map_p1(z, c); break;
            case K_MAP2_P2: el::map_p2(z, c); break;
            case K_MULT: el::mult(z, E.p0, E.ip); break;
            case K_MAP2_GEN:
              if constexpr ((kFeat & F_GEN) != 0) map_gen_call(z, c);
              break;
            case K_KQUAD:
              if constexpr ((kFeat & F_KD) != 0) el::kquad(z, c, E.ip);
              break;
            case K_CSBEND:
              if constexpr ((kFeat & F_KD) != 0) el::csbend(z, c, E.ip);
              break;
            case K_RFCA:
              if constexpr ((kFeat & F_RF) != 0) {
                const int v = p * a.nv + (E.vslot - a.v0);
                el::rfca(z, E.p0, E.p1, E.p2, a.vc[v][0], a.vc[v][1]);
              }
              break;
            case K_WAKE:
              if constexpr ((kFeat & F_WAKE) != 0) {
                const int v = p * a.nv + (E.vslot - a.v0);
                const double vs =
                    el::wake_interp(z[4], a.wake_par[0], a.wake_par[1], a.wake_v, E.ip);
                z[5] = fma(-a.vc[v][0], vs, z[5]);
              }
              break;
            case K_RADKICK:
              if constexpr ((kFeat & F_RNG) != 0) radkick_call(z[5], E.p0, pid, gp, a.seed_lo, a.seed_hi);
              break;
            default: break;
          }
          if (E.aper != TRK_APER_NONE && el::aperture_lost(E.aper, E.a0, E.a1, z)) {
            alive = false;
            rec = static_cast<int64_t>((static_cast<uint64_t>(gp) << 32) | static_cast<uint32_t>(e));
          }
        }
      }
      if constexpr (kMom) {
        double d[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) d[k] = alive ? z[k] - a.mom_shift[k] : 0.0;
        double *row = a.mom_part + (static_cast<int64_t>(p) * gridDim.x + blockIdx.x) * 28;
        block_moment_row(alive ? 1.0 : 0.0, d, row);
      }
    }
    if (act) {
#pragma unroll
      for (int k = 0; k < 6; ++k)
        if ((a.stmask >> k) & 1u) a.z[k][i] = z[k];
      if (rec >= 0) a.lost_at[i] = rec;
      if (alive) {
        smin = fmin(smin, z[4]);
        smax = fmax(smax, z[4]);
      }
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

template <uint32_t kFeat>
void launch_feat(const RunArgs &a, int grid, hipStream_t st) {
  if (a.mom)
    hipLaunchKernelGGL((k_run<kFeat, true>), dim3(grid), dim3(kBlock), 0, st, a);
  else
    hipLaunchKernelGGL((k_run<kFeat, false>), dim3(grid), dim3(kBlock), 0, st, a);
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
