// api.cpp -- host side of the C-ABI (include/trk.h): argument checks, lattice
// compilation (element classification and per-element constants), launch
// planning and sequencing.  Every step of the tracking runs in the kernels of
// the .hip translation units; nothing here touches particle data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "host.h"
#include "trk_internal.h"

using namespace trk;

namespace trk {
thread_local KernelEvents g_kernel_events{nullptr, nullptr};

namespace host {

thread_local std::string g_err;

int fail(int status, const std::string &msg) {
  g_err = msg;
  return status;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(TRK_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}


// A pointer is accepted as "device" if the runtime knows it as device or
// managed memory; plain host memory is rejected before any launch.
int check_dev(const void *p, const char *name) {
  if (p == nullptr) return fail(TRK_EINVAL, std::string(name) + " is NULL");
  hipPointerAttribute_t at;
  std::memset(&at, 0, sizeof at);
  hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(TRK_EPTR, std::string(name) + " is not a device pointer");
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
    return fail(TRK_EPTR, std::string(name) + " is not a device pointer");
  return TRK_OK;
}

int check_beam(const trk_beam *b) {
  if (b == nullptr) return fail(TRK_EINVAL, "beam is NULL");
  if (b->n_total < 0 || b->n_total > 0xffffffffLL)
    return fail(TRK_ERANGE, "n_total must lie in [0, 2^32)");
  const void *ptrs[9] = {b->x, b->xp, b->y, b->yp, b->s, b->dp, b->id, b->lost_at, b->n_alive};
  const char *names[9] = {"beam.x", "beam.xp", "beam.y", "beam.yp", "beam.s",
                          "beam.dp", "beam.id", "beam.lost_at", "beam.n_alive"};
  for (int k = 0; k < 9; ++k) {
    int r = check_dev(ptrs[k], names[k]);
    if (r) return r;
  }
  return TRK_OK;
}

int check_ws(void *ws, size_t bytes, int64_t n_total) {
  const size_t need = workspace_bytes(n_total);
  if (bytes < need) {
    char buf[128];
    std::snprintf(buf, sizeof buf, "workspace too small: %zu < %zu bytes", bytes, need);
    return fail(TRK_ERANGE, buf);
  }
  return check_dev(ws, "workspace");
}

void beam_ptrs(const trk_beam *b, double *z[6]) {
  z[0] = b->x;
  z[1] = b->xp;
  z[2] = b->y;
  z[3] = b->yp;
  z[4] = b->s;
  z[5] = b->dp;
}

}  // namespace host
}  // namespace trk

using namespace trk::host;

namespace {

// ------------------------------------------------------------------ profiling
struct Prof {
  std::mutex mu;
  uint32_t mask = 0;  // bit c: class c is timed
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[4];
  double ms[4] = {0, 0, 0, 0};
  int64_t launches[4] = {0, 0, 0, 0};
} g_prof;

// While class cls is timed, the launch's one kernel goes out through the
// extended launch with a pair of events that its dispatch packet records
// (TRK_LAUNCH); a launch that enqueued nothing leaves the pair unused.
template <class F>
hipError_t profiled(int cls, hipStream_t st, F &&launch) {
  (void)st;
  bool on;
  {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    on = ((g_prof.mask >> cls) & 1u) != 0;
  }
  if (!on) return launch();
  hipEvent_t a, b;
  hipError_t e = hipEventCreate(&a);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&b);
  if (e != hipSuccess) {
    (void)hipEventDestroy(a);
    return e;
  }
  g_kernel_events = KernelEvents{a, b};
  e = launch();
  const bool used = g_kernel_events.start == nullptr;
  g_kernel_events = KernelEvents{nullptr, nullptr};
  if (!used || e != hipSuccess) {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return e;
  }
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.ev[cls].push_back({a, b});
  return e;
}

}  // namespace

namespace trk {
namespace host {
hipError_t profiled_call(int cls, hipStream_t st, const std::function<hipError_t()> &launch) {
  return profiled(cls, st, launch);
}
}  // namespace host
}  // namespace trk

namespace {

// ------------------------------------------------------------------ constants
// Fourth-order symmetric composition (Yoshida 1990): kicks c, drifts d.
void yoshida(double c[4], double d[3]) {
  const double cr = 0x1.428a2f98d728bp+0;  // 2^(1/3), correctly rounded binary64
  const double w1 = 1.0 / (2.0 - cr);
  const double w0 = -cr / (2.0 - cr);
  c[0] = 0.5 * w1;
  c[1] = 0.5 * (w0 + w1);
  c[2] = 0.5 * (w0 + w1);
  c[3] = 0.5 * w1;
  d[0] = w1;
  d[1] = w0;
  d[2] = w1;
}

int pair_index(int j, int k) {  // (j,k), j<=k, among the 21 monomials
  return j * 6 - j * (j - 1) / 2 + (k - j);
}

// Thick quadrupole, second order: paraxial x'' = -K x, y'' = K y with
// K = k1/(1+delta).  First order cos/sin (cosh/sinh); T_ij6 = dR_ij/ddelta;
// T_5jk from the path integral of (x'^2 + y'^2)/2 along the linear orbit.
void quad_coef(double L, double k1, double c[168]) {
  std::memset(c, 0, 168 * sizeof(double));
  double *R = c + 6, *T = c + 42;
  R[4 * 6 + 4] = 1.0;
  R[5 * 6 + 5] = 1.0;
  if (k1 == 0.0) {
    R[0] = 1.0; R[1] = L; R[7] = 1.0;
    R[14] = 1.0; R[15] = L; R[21] = 1.0;
    T[4 * 21 + pair_index(1, 1)] = 0.5 * L;
    T[4 * 21 + pair_index(3, 3)] = 0.5 * L;
    return;
  }
  const double w = std::sqrt(std::fabs(k1));
  const double phi = w * L;
  const double cf = std::cos(phi), sf = std::sin(phi), s2f = std::sin(2.0 * phi);
  const double ch = std::cosh(phi), sh = std::sinh(phi), sh2 = std::sinh(2.0 * phi);
  // plane blocks: R (11 12 21 22), T (16 26 for row 1, 16 26 for row 2), S (11 12 22)
  const double foc_R[4] = {cf, sf / w, -w * sf, cf};
  const double foc_T[4] = {(0.5 * phi) * sf, (sf - phi * cf) / (2.0 * w),
                           (0.5 * w) * (sf + phi * cf), (0.5 * phi) * sf};
  const double foc_S[3] = {(0.5 * (w * w)) * (0.5 * L - s2f / (4.0 * w)), -0.5 * (sf * sf),
                           0.5 * (0.5 * L + s2f / (4.0 * w))};
  const double def_R[4] = {ch, sh / w, w * sh, ch};
  const double def_T[4] = {-((0.5 * phi) * sh), (sh - phi * ch) / (2.0 * w),
                           -((0.5 * w) * (sh + phi * ch)), -((0.5 * phi) * sh)};
  const double def_S[3] = {(0.5 * (w * w)) * (sh2 / (4.0 * w) - 0.5 * L), 0.5 * (sh * sh),
                           0.5 * (0.5 * L + sh2 / (4.0 * w))};
  for (int plane = 0; plane < 2; ++plane) {
    const bool focusing = (plane == 0) == (k1 > 0.0);
    const double *pr = focusing ? foc_R : def_R;
    const double *pt = focusing ? foc_T : def_T;
    const double *ps = focusing ? foc_S : def_S;
    const int o = 2 * plane;
    R[(o + 0) * 6 + (o + 0)] = pr[0];
    R[(o + 0) * 6 + (o + 1)] = pr[1];
    R[(o + 1) * 6 + (o + 0)] = pr[2];
    R[(o + 1) * 6 + (o + 1)] = pr[3];
    T[(o + 0) * 21 + pair_index(o, 5)] = pt[0];
    T[(o + 0) * 21 + pair_index(o + 1, 5)] = pt[1];
    T[(o + 1) * 21 + pair_index(o, 5)] = pt[2];
    T[(o + 1) * 21 + pair_index(o + 1, 5)] = pt[3];
    T[4 * 21 + pair_index(o, o)] = ps[0];
    T[4 * 21 + pair_index(o, o + 1)] = ps[1];
    T[4 * 21 + pair_index(o + 1, o + 1)] = ps[2];
  }
}

// index of z_j z_k z_l (j <= k <= l) among the 56 cubic monomials, lexicographic
int triple_index(int j, int k, int l) {
  int n = 0;
  for (int a = 0; a < 6; ++a)
    for (int b = a; b < 6; ++b)
      for (int q = b; q < 6; ++q, ++n)
        if (a == j && b == k && q == l) return n;
  return -1;
}

// Thick quadrupole to third order in the same paraxial model: the 168
// coefficients above, then the chromatic cubic terms U[6][56]:
// U_ij66 = (1/2) d^2 R_ij/d delta^2 and U_5jk6 = d T_5jk/d delta, with
// phi = omega L, omega^2 = |k1|/(1+delta), so dphi/ddelta = -phi/2 and
// d^2phi/ddelta^2 = 3 phi/4 at delta = 0.
void quad3_coef(double L, double k1, double c[504]) {
  std::memset(c, 0, 504 * sizeof(double));
  quad_coef(L, k1, c);
  if (k1 == 0.0) return;
  double *U = c + 168;
  const double w = std::sqrt(std::fabs(k1));
  const double f = w * L, f2 = f * f;
  const double cf = std::cos(f), sf = std::sin(f), c2 = std::cos(2.0 * f), s2 = std::sin(2.0 * f);
  const double ch = std::cosh(f), sh = std::sinh(f), ch2 = std::cosh(2.0 * f),
               sh2 = std::sinh(2.0 * f);
  // per plane: U of R (11 12 21 22) and of T5 (11 12 22)
  const double foc_U[4] = {-(f2 / 8.0) * cf - (3.0 * f / 8.0) * sf,
                           ((f * cf - sf) - f2 * sf) / (8.0 * w),
                           -(w / 8.0) * ((5.0 * f * cf + 3.0 * sf) - f2 * sf),
                           -(f2 / 8.0) * cf - (3.0 * f / 8.0) * sf};
  const double foc_S[3] = {-(w / 16.0) * ((4.0 * f - s2) - 2.0 * f * c2), (f * s2) / 4.0,
                           -(2.0 * f * c2 - s2) / (16.0 * w)};
  const double def_U[4] = {(f2 / 8.0) * ch + (3.0 * f / 8.0) * sh,
                           ((f2 * sh + f * ch) - sh) / (8.0 * w),
                           (w / 8.0) * ((5.0 * f * ch + 3.0 * sh) + f2 * sh),
                           (f2 / 8.0) * ch + (3.0 * f / 8.0) * sh};
  const double def_S[3] = {-(w / 16.0) * ((sh2 + 2.0 * f * ch2) - 4.0 * f), -(f * sh2) / 4.0,
                           -(2.0 * f * ch2 - sh2) / (16.0 * w)};
  for (int plane = 0; plane < 2; ++plane) {
    const bool focusing = (plane == 0) == (k1 > 0.0);
    const double *pu = focusing ? foc_U : def_U;
    const double *ps = focusing ? foc_S : def_S;
    const int o = 2 * plane;
    U[(o + 0) * 56 + triple_index(o, 5, 5)] = pu[0];
    U[(o + 0) * 56 + triple_index(o + 1, 5, 5)] = pu[1];
    U[(o + 1) * 56 + triple_index(o, 5, 5)] = pu[2];
    U[(o + 1) * 56 + triple_index(o + 1, 5, 5)] = pu[3];
    U[4 * 56 + triple_index(o, o, 5)] = ps[0];
    U[4 * 56 + triple_index(o, o + 1, 5)] = ps[1];
    U[4 * 56 + triple_index(o + 1, o + 1, 5)] = ps[2];
  }
}

// classification of a 168-coefficient map by its exact non-zero set
struct Term {
  int i, j, k;  // k < 0: an R term
};
const Term kP1[24] = {{0, 0, -1}, {0, 1, -1}, {0, 0, 5}, {0, 1, 5}, {1, 0, -1}, {1, 1, -1},
                      {1, 0, 5},  {1, 1, 5},  {2, 2, -1}, {2, 3, -1}, {2, 2, 5}, {2, 3, 5},
                      {3, 2, -1}, {3, 3, -1}, {3, 2, 5}, {3, 3, 5},  {4, 4, -1}, {4, 0, 0},
                      {4, 0, 1},  {4, 1, 1},  {4, 2, 2}, {4, 2, 3},  {4, 3, 3},  {5, 5, -1}};
const Term kP2[8] = {{0, 0, -1}, {1, 1, -1}, {2, 2, -1}, {3, 3, -1},
                     {4, 4, -1}, {4, 5, -1}, {5, 5, -1}, {4, 5, 5}};

int coef_index(const Term &t) {
  return t.k < 0 ? 6 + 6 * t.i + t.j : 42 + 21 * t.i + pair_index(t.j, t.k);
}

bool matches(const double *c, const Term *pat, int n, std::vector<double> &out) {
  std::vector<char> in_pat(168, 0);
  for (int q = 0; q < n; ++q) in_pat[coef_index(pat[q])] = 1;
  for (int q = 0; q < 168; ++q) {
    const bool nz = c[q] != 0.0;
    if (nz != static_cast<bool>(in_pat[q])) return false;
  }
  out.clear();
  for (int q = 0; q < n; ++q) out.push_back(c[coef_index(pat[q])]);
  return true;
}

// third-order maps: {i, j, k, l}, k < 0 an R term, l < 0 a T term, else U
struct Term3 {
  int i, j, k, l;
};
// the third-order thick-quad pattern: P1's 24 terms, then 14 chromatic
// cubic ones (each row's terms in evaluation order C, R, T, U)
const Term3 kP3[38] = {
    {0, 0, -1, -1}, {0, 1, -1, -1}, {0, 0, 5, -1}, {0, 1, 5, -1},
    {1, 0, -1, -1}, {1, 1, -1, -1}, {1, 0, 5, -1}, {1, 1, 5, -1},
    {2, 2, -1, -1}, {2, 3, -1, -1}, {2, 2, 5, -1}, {2, 3, 5, -1},
    {3, 2, -1, -1}, {3, 3, -1, -1}, {3, 2, 5, -1}, {3, 3, 5, -1},
    {4, 4, -1, -1}, {4, 0, 0, -1},  {4, 0, 1, -1}, {4, 1, 1, -1},
    {4, 2, 2, -1},  {4, 2, 3, -1},  {4, 3, 3, -1}, {5, 5, -1, -1},
    {0, 0, 5, 5},   {0, 1, 5, 5},   {1, 0, 5, 5},  {1, 1, 5, 5},
    {2, 2, 5, 5},   {2, 3, 5, 5},   {3, 2, 5, 5},  {3, 3, 5, 5},
    {4, 0, 0, 5},   {4, 0, 1, 5},   {4, 1, 1, 5},  {4, 2, 2, 5},
    {4, 2, 3, 5},   {4, 3, 3, 5}};

int coef_index3(const Term3 &t) {
  if (t.k < 0) return 6 + 6 * t.i + t.j;
  if (t.l < 0) return 42 + 21 * t.i + pair_index(t.j, t.k);
  return 168 + 56 * t.i + triple_index(t.j, t.k, t.l);
}

bool matches3(const double *c, const Term3 *pat, int n, std::vector<double> &out) {
  std::vector<char> in_pat(504, 0);
  for (int q = 0; q < n; ++q) in_pat[coef_index3(pat[q])] = 1;
  for (int q = 0; q < 504; ++q) {
    const bool nz = c[q] != 0.0;
    if (nz != static_cast<bool>(in_pat[q])) return false;
  }
  out.clear();
  for (int q = 0; q < n; ++q) out.push_back(c[coef_index3(pat[q])]);
  return true;
}

constexpr uint32_t M_X = 1, M_XP = 2, M_Y = 4, M_YP = 8, M_S = 16, M_DP = 32, M_ID = 64;
constexpr uint32_t M_ALL = 63;
constexpr double kStreamBytes = 256.0 * 1024 * 1024;  // MI355X Infinity Cache

}  // namespace

// ------------------------------------------------------------------ lattice

extern "C" int trk_lattice_create(const trk_element *elems, int32_t n, trk_lattice **out) {
  if (out == nullptr) return fail(TRK_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 0 || n > TRK_MAX_ELEMENTS) return fail(TRK_ERANGE, "element count out of range");
  if (n > 0 && elems == nullptr) return fail(TRK_EINVAL, "elems is NULL");
  trk_lattice *L = new (std::nothrow) trk_lattice();
  if (L == nullptr) return fail(TRK_ENOMEM, "host allocation failed");
  double yc[4], yd[3];
  yoshida(yc, yd);
  std::map<std::vector<uint64_t>, int32_t> pool_seen;
  for (int e = 0; e < n; ++e) {
    const trk_element &s = elems[e];
    DevElem d;
    std::memset(&d, 0, sizeof d);
    d.vslot = -1;
    d.off = static_cast<int32_t>(L->pool.size());
    uint32_t rd = 0, wr = 0;
    auto bad = [&](const char *why) {
      delete L;
      char buf[160];
      std::snprintf(buf, sizeof buf, "element %d: %s", e, why);
      return fail(TRK_EINVAL, buf);
    };
    switch (s.kind) {
      case TRK_EDRIFT:
        d.kind = K_EDRIFT;
        d.p0 = s.L;
        rd = M_X | M_XP | M_Y | M_YP | M_S;
        wr = M_X | M_Y | M_S;
        break;
      case TRK_QUAD:
      case TRK_MAP2:
      case TRK_MAP3: {
        double c[504];
        std::memset(c, 0, sizeof c);
        const bool third = s.kind == TRK_MAP3 || (s.kind == TRK_QUAD && s.order == 3);
        if (s.kind == TRK_QUAD) {
          if (!(s.L > 0.0)) return bad("QUAD needs L > 0");
          if (s.order != 0 && s.order != 1 && s.order != 2 && s.order != 3)
            return bad("QUAD order must be 0..3");
          if (third)
            quad3_coef(s.L, s.k, c);
          else
            quad_coef(s.L, s.k, c);
        } else {
          if (s.coef == nullptr) return bad("MAP2/MAP3 needs coef");
          std::memcpy(c, s.coef, (third ? 504 : 168) * sizeof(double));
        }
        std::vector<double> v;
        if (third) {
          if (matches3(c, kP3, 38, v)) {
            d.kind = K_MAP3_P3;
          } else {
            d.kind = K_MAP3_GEN;
            v.assign(c, c + 504);
          }
        } else if (matches(c, kP1, 24, v)) {
          d.kind = K_MAP2_P1;
        } else if (matches(c, kP2, 8, v)) {
          d.kind = K_MAP2_P2;
        } else {
          d.kind = K_MAP2_GEN;
          v.assign(c, c + 168);
        }
        L->pool.insert(L->pool.end(), v.begin(), v.end());
        // rows that are exact identities (only R_ii = 1) neither read nor write
        for (int i = 0; i < 6; ++i) {
          bool ident = c[6 + 7 * i] == 1.0 && c[i] == 0.0;
          for (int q = 0; q < 6 && ident; ++q)
            if (q != i && c[6 + 6 * i + q] != 0.0) ident = false;
          for (int q = 0; q < 21 && ident; ++q)
            if (c[42 + 21 * i + q] != 0.0) ident = false;
          for (int q = 0; q < 56 && ident; ++q)
            if (c[168 + 56 * i + q] != 0.0) ident = false;
          if (ident) continue;
          wr |= 1u << i;
          for (int j = 0; j < 6; ++j)
            if (c[6 + 6 * i + j] != 0.0) rd |= 1u << j;
          int q = 0;
          for (int j = 0; j < 6; ++j)
            for (int k = j; k < 6; ++k, ++q)
              if (c[42 + 21 * i + q] != 0.0) rd |= (1u << j) | (1u << k);
          q = 0;
          for (int j = 0; j < 6; ++j)
            for (int k = j; k < 6; ++k)
              for (int l = k; l < 6; ++l, ++q)
                if (c[168 + 56 * i + q] != 0.0) rd |= (1u << j) | (1u << k) | (1u << l);
        }
        break;
      }
      case TRK_MULT: {
        if (s.order < 1 || s.order > 8) return bad("MULT order must be 1..8");
        double f = 1.0;
        for (int i = 2; i <= s.order; ++i) f *= static_cast<double>(i);
        d.kind = K_MULT;
        d.ip = s.order;
        d.p0 = s.k / f;
        rd = M_X | M_XP | M_Y | M_YP | M_DP;
        wr = M_XP | M_YP;
        break;
      }
      case TRK_KQUAD:
      case TRK_CSBEND: {
        if (s.nsteps < 1 || s.nsteps > 4096) return bad("nsteps must be 1..4096");
        if (s.L == 0.0) return bad("kick-drift element needs L != 0");
        const double ls = s.L / static_cast<double>(s.nsteps);
        double dl[3];
        for (int i = 0; i < 3; ++i) dl[i] = yd[i] * ls;
        d.ip = s.nsteps;
        if (s.kind == TRK_KQUAD) {
          d.kind = K_KQUAD;
          for (int i = 0; i < 4; ++i) L->pool.push_back((yc[i] * ls) * s.k);
          for (int i = 0; i < 3; ++i) L->pool.push_back(dl[i]);
        } else {
          if (s.angle == 0.0) return bad("CSBEND needs angle != 0");
          d.kind = K_CSBEND;
          const double h = s.angle / s.L;
          const double rho = s.L / s.angle;
          double kA[4], kB[4];
          for (int i = 0; i < 4; ++i) {
            kA[i] = (yc[i] * ls) * h;
            kB[i] = kA[i] * h;
          }
          double cph[3], sph[3], vers[3], rs[3];
          for (int i = 0; i < 3; ++i) {
            const double phi = dl[i] * h;
            const double shalf = std::sin(0.5 * phi);
            cph[i] = std::cos(phi);
            sph[i] = std::sin(phi);
            vers[i] = 2.0 * rho * (shalf * shalf);
            rs[i] = rho * sph[i];
          }
          L->pool.insert(L->pool.end(), kA, kA + 4);
          L->pool.insert(L->pool.end(), kB, kB + 4);
          L->pool.insert(L->pool.end(), cph, cph + 3);
          L->pool.insert(L->pool.end(), sph, sph + 3);
          L->pool.insert(L->pool.end(), vers, vers + 3);
          L->pool.insert(L->pool.end(), rs, rs + 3);
          L->pool.insert(L->pool.end(), dl, dl + 3);
        }
        rd = M_ALL;
        wr = M_X | M_XP | M_Y | M_YP | M_S;
        break;
      }
      case TRK_RFCA: {
        constexpr double kTwoPi = 0x1.921fb54442d18p+2;
        d.kind = K_RFCA;
        d.p0 = 0.5 * ((kTwoPi * s.freq) / 299792458.0);
        d.p1 = std::sin(s.phase);
        d.p2 = std::cos(s.phase);
        d.p3 = s.volt;
        d.vslot = L->nvar++;
        rd = M_S | M_DP;
        wr = M_DP;
        break;
      }
      case TRK_WAKE:
        if (s.nbins < 2 || s.nbins > TRK_MAX_BINS) return bad("WAKE nbins must be 2..TRK_MAX_BINS");
        if (!(s.wake_tau0 > 0.0)) return bad("WAKE needs tau0 > 0");
        d.kind = K_WAKE;
        d.ip = s.nbins;
        d.vslot = L->nvar++;
        L->has_wake = true;
        L->max_bins = std::max(L->max_bins, s.nbins);
        rd = M_S | M_DP;
        wr = M_DP;
        break;
      case TRK_TRWAKE:
        if (s.nbins < 2 || s.nbins > TRK_MAX_TRBINS)
          return bad("TRWAKE nbins must be 2..TRK_MAX_TRBINS");
        if (!(s.wake_tau0 > 0.0)) return bad("TRWAKE needs tau0 > 0");
        d.kind = K_TRWAKE;
        d.ip = s.nbins;
        d.vslot = L->nvar++;
        L->has_wake = true;
        L->max_bins = std::max(L->max_bins, s.nbins);
        rd = M_XP | M_YP | M_S | M_DP;
        wr = M_XP | M_YP;
        break;
      case TRK_RADKICK:
        d.kind = K_RADKICK;
        d.p0 = s.sigma;
        rd = M_DP | M_ID;
        wr = M_DP;
        break;
      case TRK_MARKER:
        d.kind = K_MARKER;
        break;
      default:
        return bad("unknown element kind");
    }
    d.aper = s.aperture;
    if (s.aperture == TRK_APER_RECT) {
      if (!(s.ax > 0.0 && s.ay > 0.0)) return bad("aperture needs ax, ay > 0");
      d.a0 = s.ax;
      d.a1 = s.ay;
      rd |= M_X | M_Y;
    } else if (s.aperture == TRK_APER_ELLIPSE) {
      if (!(s.ax > 0.0 && s.ay > 0.0)) return bad("aperture needs ax, ay > 0");
      d.a0 = 1.0 / s.ax;
      d.a1 = 1.0 / s.ay;
      rd |= M_X | M_Y;
    } else if (s.aperture != TRK_APER_NONE) {
      return bad("unknown aperture");
    }
    // elements with bit-identical constants share one copy in the pool: the
    // run kernel reads them with scalar loads, and a small pool stays in
    // the scalar cache (a ring's 80 identical bends, 2 kinds of quadrupole)
    if (L->pool.size() > static_cast<size_t>(d.off)) {
      std::vector<uint64_t> key(L->pool.size() - d.off);
      std::memcpy(key.data(), L->pool.data() + d.off, key.size() * sizeof(uint64_t));
      auto it = pool_seen.find(key);
      if (it != pool_seen.end()) {
        L->pool.resize(d.off);
        d.off = it->second;
      } else {
        pool_seen.emplace(std::move(key), d.off);
      }
    }
    L->rec.push_back(d);
    trk_element cp = s;
    cp.coef = nullptr;
    L->src.push_back(cp);
    L->rd.push_back(rd);
    L->wr.push_back(wr);
    L->aper.push_back(s.aperture != TRK_APER_NONE);
    L->vslot.push_back(d.vslot);
  }
  if (L->pool.empty()) L->pool.push_back(0.0);
  size_t rb = std::max<size_t>(1, L->rec.size()) * sizeof(DevElem);
  hipError_t e = hipMalloc(&L->d_rec, rb);
  if (e == hipSuccess) e = hipMalloc(&L->d_pool, L->pool.size() * sizeof(double));
  if (e == hipSuccess && !L->rec.empty())
    e = hipMemcpy(L->d_rec, L->rec.data(), L->rec.size() * sizeof(DevElem), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(L->d_pool, L->pool.data(), L->pool.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(L->d_rec);
    (void)hipFree(L->d_pool);
    delete L;
    return fail(e == hipErrorOutOfMemory ? TRK_ENOMEM : TRK_EHIP,
                std::string("lattice upload: ") + hipGetErrorString(e));
  }
  *out = L;
  return TRK_OK;
}

extern "C" void trk_lattice_destroy(trk_lattice *lat) {
  if (lat == nullptr) return;
  (void)hipFree(lat->d_rec);
  (void)hipFree(lat->d_pool);
  delete lat;
}

// ------------------------------------------------------------------ workspace
namespace trk {

constexpr int kMomPassesMax = 16;

namespace {
struct Carver {
  char *base;
  size_t off = 0;
  template <class T>
  T *take(size_t count) {
    off = (off + 255) & ~static_cast<size_t>(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

Workspace carve(void *base, int64_t n_total, size_t *bytes) {
  const size_t n = static_cast<size_t>(std::max<int64_t>(n_total, 1));
  const size_t nb = static_cast<size_t>(std::max<int64_t>(nblocks(n_total), 1));
  Carver c{static_cast<char *>(base)};
  Workspace w;
  w.mm_part = c.take<double>(2 * std::max<size_t>(nb, kMaxRunGrid));
  w.counts = c.take<uint32_t>(TRK_MAX_BINS + 64 + 4 * TRK_MAX_TRBINS);
  w.dip = base ? reinterpret_cast<int64_t *>(w.counts + TRK_MAX_BINS + 64) : nullptr;
  w.lost_flag = c.take<uint32_t>((n + 63) / 64);
  w.range = c.take<double>(2);
  for (int k = 0; k < 2; ++k) w.hcounts[k] = c.take<uint32_t>(kHistCopies * TRK_MAX_BINS);
  w.wake_par = c.take<double>(2);
  w.wake_v = c.take<double>(2 * TRK_MAX_BINS);
  w.mom_shift = c.take<double>(6);
  w.mom_tmp = c.take<double>(28);
  w.mom_part = c.take<double>(static_cast<size_t>(kMomPassesMax) * std::max<size_t>(nb, 1024) * 28);
  w.cmp_blk = c.take<int64_t>(nb * 10);
  const size_t ct = static_cast<size_t>(std::max<int64_t>(compact_tiles(n_total), 1));
  w.rs_cnt = c.take<uint32_t>(256 * ct);
  w.rs_tot = c.take<uint32_t>(256);
  w.cmp_hdr = c.take<int64_t>(16);
  w.key_a = c.take<uint64_t>(n);
  w.key_b = c.take<uint64_t>(n);
  w.pos_a = c.take<uint32_t>(n);
  w.pos_b = c.take<uint32_t>(n);
  for (int k = 0; k < 6; ++k) w.tz[k] = c.take<double>(n);
  w.tid = c.take<uint32_t>(n);
  w.tlost = c.take<int64_t>(n);
  w.sort_tmp_bytes = sortkey_temp_bytes(static_cast<int64_t>(n));
  w.sort_tmp = c.take<char>(w.sort_tmp_bytes);
  if (bytes) *bytes = c.off + 256;
  return w;
}
}  // namespace

size_t workspace_bytes(int64_t n_total) {
  size_t b = 0;
  carve(nullptr, n_total, &b);
  return b;
}
Workspace carve_workspace(void *base, int64_t n_total) { return carve(base, n_total, nullptr); }

}  // namespace trk

extern "C" size_t trk_workspace_size(const trk_lattice *lat, int64_t n_total) {
  (void)lat;
  return workspace_bytes(n_total);
}

namespace {

bool is_wake(int32_t kind) { return kind == TRK_WAKE || kind == TRK_TRWAKE; }

// words of the counts region to clear before a histogram: the counts, and
// for a transverse wake the dipole sums that follow them
int zero_words(bool transverse) {
  return transverse ? TRK_MAX_BINS + 64 + 4 * TRK_MAX_TRBINS : TRK_MAX_BINS;
}

int grid_stride_blocks(int64_t n_total) {
  const int64_t nb = nblocks(n_total);
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(nb, kMaxGridStride)));
}

struct Launch {
  int pass0, npass, e0, e1;
};

}  // namespace

// ------------------------------------------------------------------ track
extern "C" int trk_track(trk_beam *beam, const trk_lattice *lat, int32_t passes,
                         const trk_opts *opts, void *workspace, size_t workspace_bytes_,
                         void *stream) {
  return trk::host::track_impl(beam, lat, passes, opts, workspace, workspace_bytes_, stream, true);
}

int trk::host::track_impl(trk_beam *beam, const trk_lattice *lat, int32_t passes,
                          const trk_opts *opts, void *workspace, size_t workspace_bytes_,
                          void *stream, bool compact_end) {
  if (lat == nullptr || opts == nullptr) return fail(TRK_EINVAL, "lattice or opts is NULL");
  if (passes < 0) return fail(TRK_EINVAL, "passes < 0");
  if (opts->wake_mode != TRK_WAKE_FP64 && opts->wake_mode != TRK_WAKE_FP32_MFMA)
    return fail(TRK_EINVAL, "unknown wake_mode");
  if (int r = check_beam(beam)) return r;
  if (int r = check_ws(workspace, workspace_bytes_, beam->n_total)) return r;
  if (opts->moments != nullptr)
    if (int r = check_dev(opts->moments, "opts.moments")) return r;
  const int nelem = static_cast<int>(lat->rec.size());
  if (passes == 0 || nelem == 0 || beam->n_total == 0) return TRK_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace w = carve_workspace(workspace, beam->n_total);
  double *z[6];
  beam_ptrs(beam, z);
  const bool mom = opts->moments != nullptr;

  // pass-varying constants: reference momentum through the RF cavities
  std::vector<double> vconst(static_cast<size_t>(passes) * std::max(lat->nvar, 1) * 2, 0.0);
  {
    double P = opts->p_ref_eV;
    for (int p = 0; p < passes; ++p)
      for (int e = 0; e < nelem; ++e) {
        const trk_element &s = lat->src[e];
        const int v = lat->vslot[e];
        if (s.kind == TRK_RFCA) {
          const double pn = P + s.volt * std::cos(s.phase);
          vconst[2 * (static_cast<size_t>(p) * lat->nvar + v)] = P;
          vconst[2 * (static_cast<size_t>(p) * lat->nvar + v) + 1] = 1.0 / pn;
          P = pn;
        } else if (s.kind == TRK_WAKE || s.kind == TRK_TRWAKE) {
          const double kfac = ((s.charge / static_cast<double>(beam->n_total)) * s.wake_A) / P;
          vconst[2 * (static_cast<size_t>(p) * lat->nvar + v)] = kfac;
        }
      }
  }

  // launch plan
  std::vector<Launch> plan;
  const int max_e = opts->max_elems_per_launch > 0 ? opts->max_elems_per_launch : nelem;
  // whole passes per launch: particles lost in one launch are compacted
  // away before the next (a launch of several passes costs far more than a
  // compaction, and later launches then skip the lost slots' waves)
  const bool whole_passes = !lat->has_wake && max_e >= nelem;
  auto nvar_in = [&](int e0, int e1) {
    int c = 0;
    for (int e = e0; e < e1; ++e) c += lat->vslot[e] >= 0;
    return c;
  };
  if (whole_passes) {
    int ppl = opts->passes_per_launch > 0 ? opts->passes_per_launch : 16;
    ppl = std::min(ppl, mom ? kMomPassesMax : kMaxPassesPerLaunch);
    if (lat->nvar > 0) ppl = std::min(ppl, std::max(1, kMaxVar / lat->nvar));
    if (lat->nvar > kMaxVar) return fail(TRK_ERANGE, "too many RF cavities in one lattice run");
    for (int p = 0; p < passes; p += ppl) plan.push_back({p, std::min(ppl, passes - p), 0, nelem});
  } else {
    for (int p = 0; p < passes; ++p) {
      int e0 = 0;
      while (e0 < nelem) {
        int e1 = e0 + 1;
        // extend up to the next wake, the element limit and the constant slots
        while (e1 < nelem && !is_wake(lat->src[e1].kind) && e1 - e0 < max_e &&
               nvar_in(e0, e1 + 1) <= kMaxVar)
          ++e1;
        plan.push_back({p, 1, e0, e1});
        e0 = e1;
      }
    }
  }

  if (mom) {
    // shift for the fused one-pass moments: the mean at entry
    const int g = static_cast<int>(std::min<int64_t>(nblocks(beam->n_total), 1024));
    HIP_TRY(launch_mom_partial(z, beam->n_alive, beam->n_total, nullptr, w.mom_part, g, st),
            "moments");
    HIP_TRY(launch_mom_finalize(w.mom_part, g, 1, nullptr, w.mom_tmp, 28, w.mom_shift, st),
            "moments");
  }

  int prev_mm_n = 0;  // > 0: the previous launch left (min, max) partials
  // Compaction is lazy: particles lost in a run keep their slots (the run
  // kernel skips them by their loss record) until a histogram needs the
  // alive set packed, the next launch of a whole-pass plan begins, or the
  // call ends.  The final layout does not depend on when compaction runs.
  bool dirty = false;
  // A run that changes neither s nor the alive set (RF, wake, transverse-wake
  // and random energy kicks, markers; no apertures) bins the histogram of a
  // longitudinal wake that follows it, over the range of the last histogram:
  // nothing since has moved s or lost a particle, so that range is the
  // beam's (exactly).
  // range_ok: w.range describes the current beam; fused_buf: the buffer the
  // previous run binned the coming wake's histogram into (-1: none); hnext:
  // the buffer the next such run bins into (the two alternate, so a
  // convolution can read one while clearing the other).
  bool range_ok = false;
  int fused_buf = -1, hnext = 0;
  for (size_t li = 0; li < plan.size(); ++li) {
    const Launch &L = plan[li];
    const bool starts_wake = is_wake(lat->src[L.e0].kind);
    // does the next launch start with a wake?
    bool next_wake = false, next_tr = false;
    int next_nb = 0;
    if (li + 1 < plan.size()) {
      next_wake = is_wake(lat->src[plan[li + 1].e0].kind);
      next_tr = lat->src[plan[li + 1].e0].kind == TRK_TRWAKE;
      next_nb = lat->src[plan[li + 1].e0].nbins;
    }
    const bool lmom = mom && L.e1 == nelem;
    // no element of the run moves s or loses particles (energy kicks,
    // transverse wake kicks, random energy kicks, markers; no apertures)
    bool s_fixed = true;
    for (int e = L.e0; e < L.e1; ++e) {
      const int k = lat->rec[e].kind;
      const bool keeps_s = k == K_RFCA || k == K_WAKE || k == K_TRWAKE || k == K_RADKICK ||
                           k == K_MARKER;
      if (!keeps_s || lat->aper[e]) s_fixed = false;
    }
    const bool fuse_hist = opts->run_hist >= 0 && next_wake && !next_tr && s_fixed && !lmom &&
                           (starts_wake || (range_ok && !dirty));
    if (starts_wake) {
      const bool tr = lat->src[L.e0].kind == TRK_TRWAKE;
      if (dirty) {
        HIP_TRY(launch_compact(z, beam->id, beam->lost_at, beam->n_alive, beam->n_total, w, st),
                "compact");
        dirty = false;
      }
      const int nb = lat->src[L.e0].nbins;
      const bool have_hist = !tr && fused_buf >= 0;
      if (!have_hist && prev_mm_n == 0) {
        prev_mm_n = grid_stride_blocks(beam->n_total);
        HIP_TRY(launch_minmax(beam->s, beam->n_alive, beam->n_total, w.mm_part, prev_mm_n, w.counts,
                              zero_words(tr), st),
                "minmax");
      }
      if (!have_hist) {
        HIP_TRY(profiled(2, st,
                         [&] {
                           return launch_histogram(beam->s, beam->n_alive, beam->n_total,
                                                   w.mm_part, prev_mm_n, nb, w.counts, w.range, st,
                                                   tr ? beam->x : nullptr, tr ? beam->y : nullptr,
                                                   tr ? w.dip : nullptr);
                         }),
                "histogram");
        range_ok = true;
      }
      // the run after this convolution bins the next histogram into
      // w.hcounts[hnext]: the convolution clears it
      uint32_t *clear = fuse_hist ? w.hcounts[hnext] : nullptr;
      const int nclear = fuse_hist ? kHistCopies * next_nb : 0;
      HIP_TRY(profiled(3, st,
                       [&] {
                         const trk_element &s = lat->src[L.e0];
                         if (tr)
                           return launch_convolve_tr(w.dip, nb, w.range, s.wake_tau0, s.wake_omega,
                                                     opts->wake_mode, w.wake_v, w.wake_par, st,
                                                     clear, nclear);
                         if (have_hist)
                           return launch_convolve(w.hcounts[fused_buf], nb, w.range, s.wake_tau0,
                                                  s.wake_omega, opts->wake_mode, w.wake_v,
                                                  w.wake_par, st, kHistCopies, clear, nclear);
                         return launch_convolve(w.counts, nb, w.range, s.wake_tau0, s.wake_omega,
                                                opts->wake_mode, w.wake_v, w.wake_par, st, 1,
                                                clear, nclear);
                       }),
              "convolve");
      fused_buf = -1;
    } else if (fuse_hist) {
      HIP_TRY(launch_zero_u32(w.hcounts[hnext], kHistCopies * next_nb, st), "histogram buffer");
    }
    RunArgs a;
    std::memset(&a, 0, sizeof a);
    for (int k = 0; k < 6; ++k) a.z[k] = z[k];
    a.id = beam->id;
    a.lost_at = beam->lost_at;
    a.n_alive = beam->n_alive;
    a.elems = lat->d_rec;
    a.pool = lat->d_pool;
    a.e0 = L.e0;
    a.e1 = L.e1;
    a.pass0 = opts->first_pass + L.pass0;
    a.npass = L.npass;
    a.seed_lo = static_cast<uint32_t>(opts->seed);
    a.seed_hi = static_cast<uint32_t>(opts->seed >> 32);
    uint32_t rd = 0, wr = 0;
    bool any_aper = false;
    int v0 = -1, nv = 0;
    uint32_t feat = 0;
    for (int e = L.e0; e < L.e1; ++e) {
      switch (lat->rec[e].kind) {
        case K_KQUAD:
        case K_CSBEND: feat |= F_KD; break;
        case K_RFCA: feat |= F_RF; break;
        case K_WAKE:
        case K_TRWAKE: feat |= F_WAKE; break;
        case K_RADKICK: feat |= F_RNG; break;
        case K_MAP2_GEN:
        case K_MAP3_GEN: feat |= F_GEN; break;
        default: break;
      }
      rd |= lat->rd[e];
      wr |= lat->wr[e];
      any_aper = any_aper || lat->aper[e];
      if (lat->vslot[e] >= 0) {
        if (v0 < 0) v0 = lat->vslot[e];
        ++nv;
      }
    }
    if (lmom) rd |= M_ALL;
    if (next_wake) rd |= M_S;
    a.feat = feat;
    a.n_total = beam->n_total;
    a.ldmask = rd | (wr & M_ALL);
    a.stmask = wr & M_ALL;
    a.v0 = v0 < 0 ? 0 : v0;
    a.nv = nv;
    for (int p = 0; p < L.npass; ++p)
      for (int j = 0; j < nv; ++j) {
        const size_t src = 2 * (static_cast<size_t>(L.pass0 + p) * lat->nvar + (a.v0 + j));
        a.vc[p * nv + j][0] = vconst[src];
        a.vc[p * nv + j][1] = vconst[src + 1];
      }
    a.wake_v = w.wake_v;
    a.wake_par = w.wake_par;
    a.mom = lmom ? 1 : 0;
    a.mom_part = w.mom_part;
    a.mom_shift = w.mom_shift;
    a.chk_lost = dirty ? 1 : 0;
    a.lost_flag = w.lost_flag;
    if (any_aper && !dirty) {
      // the first run since the call began or since the last compaction
      // that can lose particles: it raises the flags of its losses
      HIP_TRY(launch_zero_u32(w.lost_flag, static_cast<int>((beam->n_total + 63) / 64), st),
              "loss flags");
    }
    a.longit = opts->run_longit >= 0 && !lmom && !any_aper && !dirty &&
               ((a.ldmask | a.stmask) & ~(M_S | M_DP)) == 0 && (feat & ~(F_RF | F_WAKE)) == 0;
    // Stream with non-temporal accesses when the coordinates a run touches
    // exceed the 256 MB Infinity Cache: they cannot stay resident for the
    // next launch anyway.
    const double touched =
        8.0 * __builtin_popcount((a.ldmask | a.stmask) & M_ALL) * static_cast<double>(beam->n_total);
    a.nt = opts->run_nt > 0 ? 1 : (opts->run_nt < 0 ? 0 : (touched > kStreamBytes ? 1 : 0));
    const int grid = run_shape(a, beam->n_total, opts->run_ppt, opts->run_blocks);
    const bool binned = fuse_hist;
    if (binned) {
      a.hist_out = w.hcounts[hnext];
      a.hist_range = w.range;
      a.hist_nbins = next_nb;
    } else if (next_wake) {
      a.mm_part = w.mm_part;
      a.zero_buf = w.counts;
      a.zero_n = zero_words(next_tr);
    }
    HIP_TRY(profiled(0, st, [&] { return launch_run(a, grid, st); }), "run kernel");
    prev_mm_n = next_wake && !binned ? grid : 0;
    if (binned) {
      fused_buf = hnext;
      hnext ^= 1;
    }
    if (!s_fixed) range_ok = false;
    if (lmom) {
      double *out = opts->moments + static_cast<size_t>(L.pass0) * 28;
      HIP_TRY(launch_mom_finalize(w.mom_part, grid, L.npass, w.mom_shift, out, 28, nullptr, st),
              "moments");
    }
    dirty = dirty || any_aper;
    if (dirty && whole_passes && li + 1 < plan.size()) {
      HIP_TRY(launch_compact(z, beam->id, beam->lost_at, beam->n_alive, beam->n_total, w, st),
              "compact");
      dirty = false;
    }
  }
  if (dirty && compact_end)
    HIP_TRY(launch_compact(z, beam->id, beam->lost_at, beam->n_alive, beam->n_total, w, st),
            "compact");
  return TRK_OK;
}

// ------------------------------------------------------------------ collective calls
extern "C" int trk_histogram(const trk_beam *beam, int32_t nbins, double *range_dev,
                             uint32_t *counts_dev, void *workspace, size_t workspace_bytes_,
                             void *stream) {
  if (nbins < 2 || nbins > TRK_MAX_BINS) return fail(TRK_ERANGE, "nbins must be 2..TRK_MAX_BINS");
  if (int r = check_beam(beam)) return r;
  if (int r = check_dev(range_dev, "range")) return r;
  if (int r = check_dev(counts_dev, "counts")) return r;
  if (int r = check_ws(workspace, workspace_bytes_, beam->n_total)) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace w = carve_workspace(workspace, beam->n_total);
  const int g = grid_stride_blocks(beam->n_total);
  HIP_TRY(launch_minmax(beam->s, beam->n_alive, beam->n_total, w.mm_part, g, counts_dev, nbins, st),
          "minmax");
  HIP_TRY(launch_histogram(beam->s, beam->n_alive, beam->n_total, w.mm_part, g, nbins, counts_dev,
                           range_dev, st),
          "histogram");
  return TRK_OK;
}

extern "C" int trk_wake_convolve(const uint32_t *counts_dev, int32_t nbins, const double *range_dev,
                                 double tau0, double omega, int32_t mode, double *v_dev,
                                 void *stream) {
  if (nbins < 2 || nbins > TRK_MAX_BINS) return fail(TRK_ERANGE, "nbins must be 2..TRK_MAX_BINS");
  if (mode != TRK_WAKE_FP64 && mode != TRK_WAKE_FP32_MFMA) return fail(TRK_EINVAL, "unknown mode");
  if (!(tau0 > 0.0)) return fail(TRK_EINVAL, "tau0 must be > 0");
  if (int r = check_dev(counts_dev, "counts")) return r;
  if (int r = check_dev(range_dev, "range")) return r;
  if (int r = check_dev(v_dev, "v")) return r;
  HIP_TRY(launch_convolve(counts_dev, nbins, range_dev, tau0, omega, mode, v_dev, nullptr,
                          static_cast<hipStream_t>(stream)),
          "convolve");
  return TRK_OK;
}

extern "C" int trk_wake_kick(trk_beam *beam, const uint32_t *counts_dev, int32_t nbins,
                             const double *range_dev, const trk_wake *wk, double p_ref_eV,
                             int32_t mode, void *workspace, size_t workspace_bytes_, void *stream) {
  if (wk == nullptr) return fail(TRK_EINVAL, "wake is NULL");
  if (nbins < 2 || nbins > TRK_MAX_BINS) return fail(TRK_ERANGE, "nbins must be 2..TRK_MAX_BINS");
  if (mode != TRK_WAKE_FP64 && mode != TRK_WAKE_FP32_MFMA) return fail(TRK_EINVAL, "unknown mode");
  if (!(wk->tau0 > 0.0)) return fail(TRK_EINVAL, "tau0 must be > 0");
  if (int r = check_beam(beam)) return r;
  if (int r = check_dev(counts_dev, "counts")) return r;
  if (int r = check_dev(range_dev, "range")) return r;
  if (int r = check_ws(workspace, workspace_bytes_, beam->n_total)) return r;
  if (beam->n_total == 0) return TRK_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace w = carve_workspace(workspace, beam->n_total);
  HIP_TRY(launch_convolve(counts_dev, nbins, range_dev, wk->tau0, wk->omega, mode, w.wake_v,
                          w.wake_par, st),
          "convolve");
  const double kfac = ((wk->charge / static_cast<double>(beam->n_total)) * wk->A) / p_ref_eV;
  HIP_TRY(launch_wake_kick(beam->s, beam->dp, beam->n_alive, beam->n_total, w.wake_v, w.wake_par,
                           nbins, kfac, st),
          "wake kick");
  return TRK_OK;
}

extern "C" int trk_dipole_histogram(const trk_beam *beam, int32_t nbins, double *range_dev,
                                    uint32_t *counts_dev, int64_t *dipole_dev, void *workspace,
                                    size_t workspace_bytes_, void *stream) {
  if (nbins < 2 || nbins > TRK_MAX_TRBINS)
    return fail(TRK_ERANGE, "nbins must be 2..TRK_MAX_TRBINS");
  if (int r = check_beam(beam)) return r;
  if (int r = check_dev(range_dev, "range")) return r;
  if (int r = check_dev(counts_dev, "counts")) return r;
  if (int r = check_dev(dipole_dev, "dipole")) return r;
  if (int r = check_ws(workspace, workspace_bytes_, beam->n_total)) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace w = carve_workspace(workspace, beam->n_total);
  const int g = grid_stride_blocks(beam->n_total);
  HIP_TRY(launch_zero_u32(reinterpret_cast<uint32_t *>(dipole_dev), 4 * nbins, st), "zero");
  HIP_TRY(launch_minmax(beam->s, beam->n_alive, beam->n_total, w.mm_part, g, counts_dev, nbins, st),
          "minmax");
  HIP_TRY(launch_histogram(beam->s, beam->n_alive, beam->n_total, w.mm_part, g, nbins, counts_dev,
                           range_dev, st, beam->x, beam->y, dipole_dev),
          "dipole histogram");
  return TRK_OK;
}

extern "C" int trk_trwake_convolve(const int64_t *dipole_dev, int32_t nbins,
                                   const double *range_dev, double tau0, double omega,
                                   int32_t mode, double *v_dev, void *stream) {
  if (nbins < 2 || nbins > TRK_MAX_TRBINS)
    return fail(TRK_ERANGE, "nbins must be 2..TRK_MAX_TRBINS");
  if (mode != TRK_WAKE_FP64 && mode != TRK_WAKE_FP32_MFMA) return fail(TRK_EINVAL, "unknown mode");
  if (!(tau0 > 0.0)) return fail(TRK_EINVAL, "tau0 must be > 0");
  if (int r = check_dev(dipole_dev, "dipole")) return r;
  if (int r = check_dev(range_dev, "range")) return r;
  if (int r = check_dev(v_dev, "v")) return r;
  HIP_TRY(launch_convolve_tr(dipole_dev, nbins, range_dev, tau0, omega, mode, v_dev, nullptr,
                             static_cast<hipStream_t>(stream)),
          "convolve");
  return TRK_OK;
}

extern "C" int trk_trwake_kick(trk_beam *beam, const int64_t *dipole_dev, int32_t nbins,
                               const double *range_dev, const trk_wake *wk, double p_ref_eV,
                               int32_t mode, void *workspace, size_t workspace_bytes_,
                               void *stream) {
  if (wk == nullptr) return fail(TRK_EINVAL, "wake is NULL");
  if (nbins < 2 || nbins > TRK_MAX_TRBINS)
    return fail(TRK_ERANGE, "nbins must be 2..TRK_MAX_TRBINS");
  if (mode != TRK_WAKE_FP64 && mode != TRK_WAKE_FP32_MFMA) return fail(TRK_EINVAL, "unknown mode");
  if (!(wk->tau0 > 0.0)) return fail(TRK_EINVAL, "tau0 must be > 0");
  if (int r = check_beam(beam)) return r;
  if (int r = check_dev(dipole_dev, "dipole")) return r;
  if (int r = check_dev(range_dev, "range")) return r;
  if (int r = check_ws(workspace, workspace_bytes_, beam->n_total)) return r;
  if (beam->n_total == 0) return TRK_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace w = carve_workspace(workspace, beam->n_total);
  HIP_TRY(launch_convolve_tr(dipole_dev, nbins, range_dev, wk->tau0, wk->omega, mode, w.wake_v,
                             w.wake_par, st),
          "convolve");
  const double kfac = ((wk->charge / static_cast<double>(beam->n_total)) * wk->A) / p_ref_eV;
  double *z[6];
  beam_ptrs(beam, z);
  HIP_TRY(launch_trwake_kick(z, beam->n_alive, beam->n_total, w.wake_v, w.wake_par, nbins, kfac,
                             st),
          "transverse wake kick");
  return TRK_OK;
}

extern "C" int trk_moments(const trk_beam *beam, double *out_dev, void *workspace,
                           size_t workspace_bytes_, void *stream) {
  if (int r = check_beam(beam)) return r;
  if (int r = check_dev(out_dev, "out")) return r;
  if (int r = check_ws(workspace, workspace_bytes_, beam->n_total)) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace w = carve_workspace(workspace, beam->n_total);
  double *z[6];
  beam_ptrs(beam, z);
  const int g = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(nblocks(beam->n_total), 1024)));
  HIP_TRY(launch_mom_partial(z, beam->n_alive, beam->n_total, nullptr, w.mom_part, g, st), "moments");
  HIP_TRY(launch_mom_finalize(w.mom_part, g, 1, nullptr, w.mom_tmp, 28, w.mom_shift, st), "moments");
  HIP_TRY(launch_mom_partial(z, beam->n_alive, beam->n_total, w.mom_shift, w.mom_part, g, st),
          "moments");
  HIP_TRY(launch_mom_finalize(w.mom_part, g, 1, w.mom_shift, out_dev, 28, nullptr, st), "moments");
  return TRK_OK;
}

extern "C" int trk_moments_compensated(const trk_beam *beam, double *out_dev, void *workspace,
                                       size_t workspace_bytes_, void *stream) {
  if (int r = check_beam(beam)) return r;
  if (int r = check_dev(out_dev, "out")) return r;
  if (int r = check_ws(workspace, workspace_bytes_, beam->n_total)) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace w = carve_workspace(workspace, beam->n_total);
  double *z[6];
  beam_ptrs(beam, z);
  const int g = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(nblocks(beam->n_total), 1024)));
  HIP_TRY(launch_mom_partial_c(z, beam->n_alive, beam->n_total, nullptr, w.mom_part, g, st),
          "compensated moments");
  HIP_TRY(launch_mom_finalize_c(w.mom_part, g, nullptr, w.mom_tmp, w.mom_shift, st),
          "compensated moments");
  HIP_TRY(launch_mom_partial_c(z, beam->n_alive, beam->n_total, w.mom_shift, w.mom_part, g, st),
          "compensated moments");
  HIP_TRY(launch_mom_finalize_c(w.mom_part, g, w.mom_shift, out_dev, nullptr, st),
          "compensated moments");
  return TRK_OK;
}

extern "C" int trk_compact_lost_mode(trk_beam *beam, int32_t mode, void *workspace,
                                     size_t workspace_bytes_, void *stream) {
  if (mode != TRK_COMPACT_STABLE && mode != TRK_COMPACT_SWAP && mode != TRK_COMPACT_SORT)
    return fail(TRK_EINVAL, "unknown compaction mode");
  if (mode == TRK_COMPACT_STABLE)
    return trk_compact_lost(beam, workspace, workspace_bytes_, stream);
  if (int r = check_beam(beam)) return r;
  if (int r = check_ws(workspace, workspace_bytes_, beam->n_total)) return r;
  if (beam->n_total == 0) return TRK_OK;
  if (beam->n_total > 0x7fffffffLL) return fail(TRK_ERANGE, "n_total beyond 2^31 - 1");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace w = carve_workspace(workspace, beam->n_total);
  double *z[6];
  beam_ptrs(beam, z);
  HIP_TRY(launch_compact_variant(mode, z, beam->id, beam->lost_at, beam->n_alive, beam->n_total, w,
                                 st),
          "compact");
  return TRK_OK;
}

extern "C" int trk_compact_lost(trk_beam *beam, void *workspace, size_t workspace_bytes_,
                                void *stream) {
  if (int r = check_beam(beam)) return r;
  if (int r = check_ws(workspace, workspace_bytes_, beam->n_total)) return r;
  if (beam->n_total == 0) return TRK_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  Workspace w = carve_workspace(workspace, beam->n_total);
  double *z[6];
  beam_ptrs(beam, z);
  HIP_TRY(launch_compact(z, beam->id, beam->lost_at, beam->n_alive, beam->n_total, w, st),
          "compact");
  return TRK_OK;
}

// ------------------------------------------------------------------ batches
struct trk_batch {
  int nvar = 0, nelem = 0;
  uint32_t feat = 0, ldmask = 0, stmask = 0;
  std::vector<int64_t> seg_off;
  std::vector<int64_t> chunk_off[3];  // ppt 1, 2, 4
  DevElem *d_rec = nullptr;
  double *d_pool = nullptr;
  int64_t *d_seg_off = nullptr;
  int64_t *d_chunk_off[3] = {nullptr, nullptr, nullptr};
  uint64_t *d_seeds = nullptr;
  int ncu = 0;
  // cached graph of the last launch sequence, captured on a private stream
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  std::vector<uint64_t> key;
};

namespace {
int ppt_slot(int ppt) { return ppt >= 4 ? 2 : (ppt == 2 ? 1 : 0); }
int ppt_of_slot(int k) { return k == 2 ? 4 : (k == 1 ? 2 : 1); }
constexpr int kBatchMomPasses = 64;
}  // namespace

extern "C" int trk_batch_create(const trk_lattice *const *lats, int32_t nvar, const int64_t *seg_off,
                                const uint64_t *seeds, trk_batch **out) {
  if (out == nullptr) return fail(TRK_EINVAL, "out is NULL");
  *out = nullptr;
  if (nvar < 1 || lats == nullptr || seg_off == nullptr || seeds == nullptr)
    return fail(TRK_EINVAL, "need nvar >= 1 lattices, offsets and seeds");
  const int nelem = static_cast<int>(lats[0] ? lats[0]->rec.size() : 0);
  if (nelem == 0) return fail(TRK_EINVAL, "empty lattice");
  if (seg_off[0] != 0) return fail(TRK_EINVAL, "seg_off[0] must be 0");
  std::vector<DevElem> rec;
  std::vector<double> pool;
  trk_batch *B = new (std::nothrow) trk_batch();
  if (B == nullptr) return fail(TRK_ENOMEM, "host allocation failed");
  B->nvar = nvar;
  B->nelem = nelem;
  for (int v = 0; v < nvar; ++v) {
    const trk_lattice *L = lats[v];
    if (L == nullptr || static_cast<int>(L->rec.size()) != nelem) {
      delete B;
      return fail(TRK_EINVAL, "batch lattices must have equal length");
    }
    if (seg_off[v + 1] < seg_off[v]) {
      delete B;
      return fail(TRK_EINVAL, "seg_off must be non-decreasing");
    }
    const int32_t shift = static_cast<int32_t>(pool.size());
    for (int e = 0; e < nelem; ++e) {
      if (L->src[e].kind != lats[0]->src[e].kind) {
        delete B;
        return fail(TRK_EINVAL, "batch lattices must have the same element kinds");
      }
      if (L->src[e].kind == TRK_RFCA || is_wake(L->src[e].kind)) {
        delete B;
        return fail(TRK_EINVAL, "RF cavities and wakes are not supported in batches");
      }
      DevElem d = L->rec[e];
      d.off += shift;
      rec.push_back(d);
      switch (d.kind) {
        case K_KQUAD:
        case K_CSBEND: B->feat |= F_KD; break;
        case K_RADKICK: B->feat |= F_RNG; break;
        case K_MAP2_GEN:
        case K_MAP3_GEN: B->feat |= F_GEN; break;
        default: break;
      }
      B->ldmask |= L->rd[e] | L->wr[e];
      B->stmask |= L->wr[e];
    }
    pool.insert(pool.end(), L->pool.begin(), L->pool.end());
  }
  B->ldmask &= 127u;
  B->stmask &= 63u;
  B->seg_off.assign(seg_off, seg_off + nvar + 1);
  for (int k = 0; k < 3; ++k) {
    const int64_t ch = static_cast<int64_t>(kBlock) * ppt_of_slot(k);
    B->chunk_off[k].assign(nvar + 1, 0);
    for (int v = 0; v < nvar; ++v)
      B->chunk_off[k][v + 1] = B->chunk_off[k][v] + (seg_off[v + 1] - seg_off[v] + ch - 1) / ch;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&B->ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipMalloc(&B->d_rec, rec.size() * sizeof(DevElem));
  if (e == hipSuccess) e = hipMalloc(&B->d_pool, std::max<size_t>(1, pool.size()) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&B->d_seg_off, (nvar + 1) * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(&B->d_seeds, nvar * sizeof(uint64_t));
  for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipMalloc(&B->d_chunk_off[k], (nvar + 1) * sizeof(int64_t));
  if (e == hipSuccess)
    e = hipMemcpy(B->d_rec, rec.data(), rec.size() * sizeof(DevElem), hipMemcpyHostToDevice);
  if (e == hipSuccess && !pool.empty())
    e = hipMemcpy(B->d_pool, pool.data(), pool.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(B->d_seg_off, seg_off, (nvar + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(B->d_seeds, seeds, nvar * sizeof(uint64_t), hipMemcpyHostToDevice);
  for (int k = 0; k < 3 && e == hipSuccess; ++k)
    e = hipMemcpy(B->d_chunk_off[k], B->chunk_off[k].data(), (nvar + 1) * sizeof(int64_t),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    trk_batch_destroy(B);
    return fail(e == hipErrorOutOfMemory ? TRK_ENOMEM : TRK_EHIP,
                std::string("batch upload: ") + hipGetErrorString(e));
  }
  *out = B;
  return TRK_OK;
}

extern "C" void trk_batch_destroy(trk_batch *b) {
  if (b == nullptr) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  (void)hipFree(b->d_rec);
  (void)hipFree(b->d_pool);
  (void)hipFree(b->d_seg_off);
  (void)hipFree(b->d_seeds);
  for (int k = 0; k < 3; ++k) (void)hipFree(b->d_chunk_off[k]);
  delete b;
}

// Batch workspace: the ticket counter (256 B), the moment rows
// [chunks][ppl][28], the variants' moment shifts [nvar][6] and the per-chunk
// sums of the mean at entry [chunks][7] (chunks counted at one particle per
// thread, the most).
namespace {
size_t batch_mom_bytes(const trk_batch *b, int64_t ppl) {
  return static_cast<size_t>(b->chunk_off[0][b->nvar]) * ppl * 28 * sizeof(double);
}
size_t batch_shift_bytes(const trk_batch *b) {
  return (static_cast<size_t>(b->nvar) * 6 * sizeof(double) + 255) / 256 * 256;
}
}  // namespace

extern "C" size_t trk_batch_workspace_size(const trk_batch *b, int32_t passes_per_launch) {
  if (b == nullptr) return 0;
  const int64_t ppl = std::max(1, std::min<int>(passes_per_launch <= 0 ? kBatchMomPasses : passes_per_launch,
                                                kBatchMomPasses));
  return 256 + (batch_mom_bytes(b, ppl) + 255) / 256 * 256 + batch_shift_bytes(b) +
         static_cast<size_t>(b->chunk_off[0][b->nvar]) * 7 * sizeof(double) + 256;
}

namespace {
// enqueue the launches of one batched call on st
hipError_t batch_sequence(trk_batch *b, const trk_beam *beam, int passes, int first_pass,
                          const trk_batch_tuning &tu, double *moments, uint32_t *ticket,
                          double *mom_part, double *shift, double *mean_part, int ppl,
                          hipStream_t st) {
  const int k = ppt_slot(tu.ppt);
  const int grid = std::max(1, tu.blocks_per_cu) * std::max(1, b->ncu);
  BatchArgs a;
  std::memset(&a, 0, sizeof a);
  double *z[6];
  beam_ptrs(beam, z);
  for (int q = 0; q < 6; ++q) a.z[q] = z[q];
  a.id = beam->id;
  a.lost_at = beam->lost_at;
  a.seg_off = b->d_seg_off;
  a.chunk_off = b->d_chunk_off[k];
  a.seeds = b->d_seeds;
  a.elems = b->d_rec;
  a.pool = b->d_pool;
  a.nelem = b->nelem;
  a.nvar = b->nvar;
  a.ldmask = b->ldmask | (moments ? M_ALL : 0u);
  a.stmask = b->stmask;
  a.ticket = ticket;
  a.total = b->chunk_off[k][b->nvar];
  a.mom_part = moments ? mom_part : nullptr;
  a.mom_shift = shift;
  a.mean_part = mean_part;
  if (moments) {
    hipError_t e = launch_batch_mean(a, ppt_of_slot(k), st);
    if (e != hipSuccess) return e;
  }
  for (int p0 = 0; p0 < passes; p0 += ppl) {
    const int np = std::min(ppl, passes - p0);
    a.pass0 = first_pass + p0;
    a.npass = np;
    hipError_t e = launch_zero_u32(ticket, 1, st);
    if (e != hipSuccess) return e;
    e = launch_batch(a, b->feat, ppt_of_slot(k), grid, st);
    if (e != hipSuccess) return e;
    if (moments) {
      e = launch_batch_mom_finalize(mom_part, b->d_chunk_off[k], shift, b->nvar, np, moments, p0,
                                    passes, st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}
}  // namespace

extern "C" int trk_track_batched(trk_batch *b, const trk_beam *beam, int32_t passes,
                                 int32_t first_pass, const trk_batch_tuning *tune,
                                 double *moments_dev, void *workspace, size_t workspace_bytes_,
                                 void *stream) {
  if (b == nullptr || tune == nullptr) return fail(TRK_EINVAL, "batch or tuning is NULL");
  if (passes < 0) return fail(TRK_EINVAL, "passes < 0");
  if (int r = check_beam(beam)) return r;
  if (beam->n_total != b->seg_off[b->nvar])
    return fail(TRK_EINVAL, "beam.n_total must equal seg_off[nvar]");
  int ppl = tune->passes_per_launch > 0 ? tune->passes_per_launch : passes;
  if (moments_dev != nullptr) {
    if (int r = check_dev(moments_dev, "moments")) return r;
    ppl = std::min(ppl, kBatchMomPasses);
  }
  ppl = std::max(ppl, 1);
  const size_t need = trk_batch_workspace_size(b, ppl);
  if (workspace_bytes_ < need) return fail(TRK_ERANGE, "batch workspace too small");
  if (int r = check_dev(workspace, "workspace")) return r;
  if (passes == 0 || beam->n_total == 0) return TRK_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char *wsb = static_cast<char *>(workspace);
  uint32_t *ticket = reinterpret_cast<uint32_t *>(wsb);
  double *mom_part = reinterpret_cast<double *>(wsb + 256);
  const size_t mom_b = (batch_mom_bytes(b, ppl) + 255) / 256 * 256;
  double *shift = reinterpret_cast<double *>(wsb + 256 + mom_b);
  double *mean_part = reinterpret_cast<double *>(wsb + 256 + mom_b + batch_shift_bytes(b));
  if (!tune->use_graph) {
    HIP_TRY(batch_sequence(b, beam, passes, first_pass, *tune, moments_dev, ticket, mom_part, shift,
                           mean_part, ppl, st),
            "batch");
    return TRK_OK;
  }
  std::vector<uint64_t> key = {reinterpret_cast<uint64_t>(beam->x), reinterpret_cast<uint64_t>(beam->id),
                               reinterpret_cast<uint64_t>(beam->lost_at), static_cast<uint64_t>(passes),
                               static_cast<uint64_t>(static_cast<uint32_t>(first_pass)),
                               static_cast<uint64_t>(tune->ppt), static_cast<uint64_t>(tune->blocks_per_cu),
                               static_cast<uint64_t>(ppl), reinterpret_cast<uint64_t>(moments_dev),
                               reinterpret_cast<uint64_t>(workspace)};
  for (int q = 1; q < 6; ++q) key.push_back(reinterpret_cast<uint64_t>((&beam->x)[q]));
  if (b->exec == nullptr || key != b->key) {
    if (b->exec) {
      HIP_TRY(hipGraphExecDestroy(b->exec), "graph destroy");
      b->exec = nullptr;
    }
    if (b->cap == nullptr) HIP_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "stream");
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "begin capture");
    hipError_t e = batch_sequence(b, beam, passes, first_pass, *tune, moments_dev, ticket, mom_part,
                                  shift, mean_part, ppl, b->cap);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess) return hip_fail(e, "batch capture");
    if (e2 != hipSuccess) return hip_fail(e2, "end capture");
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->exec = nullptr;
      return hip_fail(e, "graph instantiate");
    }
    b->key = key;
  }
  HIP_TRY(hipGraphLaunch(b->exec, st), "graph launch");
  return TRK_OK;
}

// ------------------------------------------------------------------ test hooks
extern "C" int trk_elementary(int32_t fn, const double *x_dev, const double *y_dev, double *out_dev,
                              int64_t n, void *stream) {
  if (fn < 0 || fn > 5) return fail(TRK_EINVAL, "fn must be 0..5");
  if (n < 0) return fail(TRK_EINVAL, "n < 0");
  if (n == 0) return TRK_OK;
  if (int r = check_dev(x_dev, "x")) return r;
  if (fn == 5)
    if (int r = check_dev(y_dev, "y")) return r;
  if (int r = check_dev(out_dev, "out")) return r;
  HIP_TRY(launch_elementary(fn, x_dev, y_dev, out_dev, n, static_cast<hipStream_t>(stream)),
          "elementary");
  return TRK_OK;
}

extern "C" int trk_philox4x32_10(const uint32_t *ctr_dev, const uint32_t *key_dev,
                                 uint32_t *out_dev, int64_t n, void *stream) {
  if (n < 0) return fail(TRK_EINVAL, "n < 0");
  if (n == 0) return TRK_OK;
  if (int r = check_dev(ctr_dev, "ctr")) return r;
  if (int r = check_dev(key_dev, "key")) return r;
  if (int r = check_dev(out_dev, "out")) return r;
  HIP_TRY(launch_philox(ctr_dev, key_dev, out_dev, n, static_cast<hipStream_t>(stream)), "philox");
  return TRK_OK;
}

extern "C" int trk_gauss(const uint32_t *id_dev, uint32_t step, uint32_t tag, uint64_t seed,
                         double *out_dev, int64_t n, void *stream) {
  if (n < 0) return fail(TRK_EINVAL, "n < 0");
  if (n == 0) return TRK_OK;
  if (int r = check_dev(id_dev, "id")) return r;
  if (int r = check_dev(out_dev, "out")) return r;
  HIP_TRY(launch_gauss(id_dev, step, tag, seed, out_dev, n, static_cast<hipStream_t>(stream)),
          "gauss");
  return TRK_OK;
}

extern "C" int trk_probe_stream(const double *src_dev, double *dst_dev, int64_t n, int32_t mode,
                                int32_t blocks, void *stream) {
  if (mode < 0 || mode > 2)
    return fail(TRK_EINVAL, "mode must be 0 (copy), 1 (read) or 2 (non-temporal copy)");
  if (n < 0) return fail(TRK_EINVAL, "n < 0");
  if (blocks < 1 || blocks > (1 << 20)) return fail(TRK_EINVAL, "blocks must be 1..2^20");
  if (n == 0) return TRK_OK;
  if (int r = check_dev(src_dev, "src")) return r;
  if (int r = check_dev(dst_dev, "dst")) return r;
  HIP_TRY(launch_probe_stream(src_dev, dst_dev, n, mode, blocks, static_cast<hipStream_t>(stream)),
          "stream probe");
  return TRK_OK;
}

extern "C" int trk_probe_fma(double *out_dev, int32_t iters, int32_t blocks, void *stream) {
  if (iters < 0) return fail(TRK_EINVAL, "iters < 0");
  if (blocks < 1 || blocks > (1 << 20)) return fail(TRK_EINVAL, "blocks must be 1..2^20");
  if (int r = check_dev(out_dev, "out")) return r;
  HIP_TRY(launch_probe_fma(out_dev, iters, blocks, static_cast<hipStream_t>(stream)), "fma probe");
  return TRK_OK;
}

// ------------------------------------------------------------------ misc
extern "C" const char *trk_status_string(int status) {
  switch (status) {
    case TRK_OK: return "ok";
    case TRK_EINVAL: return "invalid argument";
    case TRK_EPTR: return "host pointer where a device pointer is required";
    case TRK_EHIP: return "HIP runtime error";
    case TRK_ENOMEM: return "out of device memory";
    case TRK_ERANGE: return "size out of range";
    default: return "unknown status";
  }
}

extern "C" const char *trk_last_error(void) { return g_err.c_str(); }

extern "C" int trk_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.mask = static_cast<uint32_t>(on) & 0xFu;
  if (on) {
    for (int c = 0; c < 4; ++c) {
      for (auto &p : g_prof.ev[c]) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
      }
      g_prof.ev[c].clear();
      g_prof.ms[c] = 0.0;
      g_prof.launches[c] = 0;
    }
  }
  return TRK_OK;
}

extern "C" int trk_profile_read(int32_t cls, double *total_ms, int64_t *launches) {
  if (cls < 0 || cls > 3 || total_ms == nullptr || launches == nullptr)
    return fail(TRK_EINVAL, "bad profile query");
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (auto &p : g_prof.ev[cls]) {
    HIP_TRY(hipEventSynchronize(p.second), "event sync");
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, p.first, p.second), "event time");
    g_prof.ms[cls] += ms;
    g_prof.launches[cls] += 1;
    (void)hipEventDestroy(p.first);
    (void)hipEventDestroy(p.second);
  }
  g_prof.ev[cls].clear();
  *total_ms = g_prof.ms[cls];
  *launches = g_prof.launches[cls];
  return TRK_OK;
}
