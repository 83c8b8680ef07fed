// scratch.hip -- the allocation-free form of trk_moments.
//
// trk_moments takes its partial sums from a caller-supplied workspace.  For
// callers that cannot allocate device memory at all (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation) the same
// two-pass reduction runs on a fixed scratch array that lives in the code
// object itself: a file-scope __device__ array, one copy per GPU, allocated
// when the library's code object is loaded onto that GPU and held until the
// process ends.
//
// In host code the array's name is only a host-side stand-in; its device
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and that address is what the kernels receive.
#include <mutex>

#include "host.h"

namespace trk {

hipError_t launch_mom_partial(double *const z[6], const int64_t *n_alive, int64_t n_total,
                              const double *shift, double *part, int grid, hipStream_t st);
hipError_t launch_mom_finalize(const double *part, int nrows, int npass, const double *shift,
                               double *out, int out_stride, double *mean_out, hipStream_t st);

namespace {

// Layout: kScratchRows partial rows of 28 doubles, then the 28-entry
// first-pass result and the 6-entry shift, each at a 256-byte boundary.
constexpr int kScratchRows = 1024;
constexpr size_t kPartBytes = static_cast<size_t>(kScratchRows) * 28 * sizeof(double);
constexpr size_t kTmpOff = (kPartBytes + 255) & ~static_cast<size_t>(255);
constexpr size_t kShiftOff = kTmpOff + 256;
constexpr size_t kScratchUsed = kShiftOff + 6 * sizeof(double);
constexpr size_t kScratchBytes = 256 * 1024;
static_assert(kScratchUsed <= kScratchBytes, "scratch layout");

__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of this GPU's scratch copy (looked up on the first call
// made with that device current)
int scratch_address(void **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return host::fail(TRK_ERANGE, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void *p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (p == nullptr) return host::fail(TRK_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TRK_OK;
}

}  // namespace
}  // namespace trk

using namespace trk;

extern "C" int trk_moments_noalloc(const trk_beam *beam, double *out_dev, void *stream) {
  if (int r = host::check_beam(beam)) return r;
  if (int r = host::check_dev(out_dev, "out")) return r;
  // the grid, and with it the scratch the reduction needs, is capped: any
  // n_total fits, and a larger request is refused rather than overrun
  const int g = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(nblocks(beam->n_total),
                                                                         kScratchRows)));
  const size_t need = kTmpOff + 256 + 6 * sizeof(double);
  if (g > kScratchRows || need > kScratchBytes)
    return host::fail(TRK_ERANGE, "moments need more than the 256 KiB static scratch");
  void *base = nullptr;
  if (int r = scratch_address(&base)) return r;
  char *b = static_cast<char *>(base);
  double *part = reinterpret_cast<double *>(b);
  double *tmp = reinterpret_cast<double *>(b + kTmpOff);
  double *shift = reinterpret_cast<double *>(b + kShiftOff);
  hipStream_t st = static_cast<hipStream_t>(stream);
  double *z[6];
  host::beam_ptrs(beam, z);
  // every scratch entry read below is written earlier in the same call
  // (g partial rows, then the 28 results and the shift), so nothing left by
  // a previous call is used and nothing needs clearing
  HIP_TRY(launch_mom_partial(z, beam->n_alive, beam->n_total, nullptr, part, g, st), "moments");
  HIP_TRY(launch_mom_finalize(part, g, 1, nullptr, tmp, 28, shift, st), "moments");
  HIP_TRY(launch_mom_partial(z, beam->n_alive, beam->n_total, shift, part, g, st), "moments");
  HIP_TRY(launch_mom_finalize(part, g, 1, shift, out_dev, 28, nullptr, st), "moments");
  return TRK_OK;
}
