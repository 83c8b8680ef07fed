// host.h -- host-side helpers shared by the C-ABI translation units
// (argument checks, error reporting) and the lattice handle.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

#include "trk_internal.h"

namespace trk {
namespace host {
int fail(int status, const std::string &msg);
int hip_fail(hipError_t e, const char *what);
// accepted: device or managed memory; plain host memory is rejected
int check_dev(const void *p, const char *name);
int check_beam(const trk_beam *b);
int check_ws(void *ws, size_t bytes, int64_t n_total);
void beam_ptrs(const trk_beam *b, double *z[6]);
// launch bracketed by HIP events while profiling is enabled (trk_profile_*);
// classes: 0 fused element run, 1 surrogate network inference, 2 wake
// histogram, 3 wake convolution
hipError_t profiled_call(int cls, hipStream_t st, const std::function<hipError_t()> &launch);

// trk_track; with compact_end false a beam that lost particles is left
// uncompacted at the end of the call (lost particles keep their slots, marked
// in lost_at), for a caller that reorders the beam itself afterwards
int track_impl(trk_beam *beam, const trk_lattice *lat, int32_t passes, const trk_opts *opts,
               void *workspace, size_t workspace_bytes, void *stream, bool compact_end);
}  // namespace host
}  // namespace trk

#define HIP_TRY(expr, what)                                \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return trk::host::hip_fail(e_, what); \
  } while (0)

struct trk_lattice {
  std::vector<trk::DevElem> rec;
  std::vector<double> pool;
  std::vector<trk_element> src;
  std::vector<uint32_t> rd, wr;   // per element coordinate masks
  std::vector<char> aper;         // element has an aperture
  std::vector<int> vslot;         // -1 or ordinal among pass-varying elements
  int nvar = 0;
  bool has_wake = false;
  int max_bins = 0;
  trk::DevElem *d_rec = nullptr;
  double *d_pool = nullptr;
};

