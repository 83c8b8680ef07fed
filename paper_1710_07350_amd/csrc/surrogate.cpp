// surrogate.cpp -- host side of the learned section surrogate (include/trk.h):
// the network handle (FP32 master weights, Adam state, bfloat16 copies), the
// training loop, and the section handle (linear map by central differences
// of the tracker, Twiss parameters and gate constants) with the calls that
// chain the gate, sampler, pairs, inference and fallback kernels.  All
// per-particle work runs in the kernels of mlp.hip and surr.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "host.h"
#include "mlp.h"

using namespace trk;
using namespace trk::host;

namespace {

constexpr double kB1 = 0.9, kB2 = 0.999, kEps = 1e-8;
constexpr double kPi = 3.14159265358979323846;
constexpr int64_t kWfElems = 256 * 32 + 256 * 256 + 256 * 256 + 16 * 256;  // w1f w2f w3f w4f
constexpr int64_t kWbElems = 256 * 32 + 256 * 256 + 256 * 256;             // w4b w3b w2b
constexpr uint16_t kBf16One = 0x3F80;

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

int check_prec(int32_t p) {
  if (p != TRK_MLP_BF16 && p != TRK_MLP_BF16X2) return fail(TRK_EINVAL, "unknown precision");
  return TRK_OK;
}

}  // namespace

// ------------------------------------------------------------------ network
struct trk_mlp {
  float *w = nullptr, *m = nullptr, *v = nullptr;  // [NPARAM] each, one allocation
  uint16_t *bf = nullptr;                          // bf16 copies, one allocation
  uint16_t *wi = nullptr;                          // inference copies
  uint16_t *w1f, *w2f, *w3f, *w4f, *w4b, *w3b, *w2b;
  int64_t step = 0;
  double p1 = 1.0, p2 = 1.0;  // beta1^step, beta2^step (products in step order)
};

namespace {

MlpDev dev_of(const trk_mlp *m) {
  MlpDev d;
  d.w1f = m->w1f;
  d.w2f = m->w2f;
  d.w3f = m->w3f;
  d.w4f = m->w4f;
  d.w4b = m->w4b;
  d.w3b = m->w3b;
  d.w2b = m->w2b;
  d.b1 = m->w + kOffB1;
  d.b2 = m->w + kOffB2;
  d.b3 = m->w + kOffB3;
  d.b4 = m->w + kOffB4;
  d.wi = m->wi;
  return d;
}

AdamArgs adam_base(trk_mlp *m) {
  AdamArgs a{};
  a.w = m->w;
  a.m = m->m;
  a.v = m->v;
  a.b1 = kB1;
  a.b2 = kB2;
  a.omb1 = 1.0 - kB1;
  a.omb2 = 1.0 - kB2;
  a.eps = kEps;
  a.w1f = m->w1f;
  a.w2f = m->w2f;
  a.w3f = m->w3f;
  a.w4f = m->w4f;
  a.w4b = m->w4b;
  a.w3b = m->w3b;
  a.w2b = m->w2b;
  a.bc1 = 1.0;
  a.bc2 = 1.0;
  return a;
}

// advance the step count and the bias-correction products
void next_step(trk_mlp *m, AdamArgs &a, double lr) {
  m->step += 1;
  m->p1 = m->p1 * kB1;
  m->p2 = m->p2 * kB2;
  a.bc1 = 1.0 - m->p1;
  a.bc2 = 1.0 - m->p2;
  a.lr = lr;
}

// training workspace for batches of B rows
struct TrainWs {
  uint16_t *uT, *hT[3], *dO, *dOT, *dAT[3];
  float *aT[3], *part[4], *loss_part;
  int slices;
  int64_t kslice;
};

int64_t kslice_of(int64_t B) { return (B % 512 == 0) ? 512 : 64; }

TrainWs carve_train(void *base, int64_t B, size_t *bytes) {
  Carver c{static_cast<char *>(base)};
  TrainWs w;
  w.kslice = kslice_of(B);
  w.slices = static_cast<int>(B / w.kslice);
  const size_t b = static_cast<size_t>(B);
  w.uT = c.take<uint16_t>(kMlpInPadT * b);
  for (int k = 0; k < 3; ++k) w.hT[k] = c.take<uint16_t>(kMlpHT * b);
  for (int k = 0; k < 3; ++k) w.aT[k] = c.take<float>(kMlpHid * b);
  w.dO = c.take<uint16_t>(kMlpInPad * b);
  w.dOT = c.take<uint16_t>(kMlpOutPad * b);
  for (int k = 0; k < 3; ++k) w.dAT[k] = c.take<uint16_t>(kMlpHid * b);
  const size_t S = static_cast<size_t>(w.slices);
  w.part[0] = c.take<float>(S * kMlpHid * kMlpInPadT);
  w.part[1] = c.take<float>(S * kMlpHid * kMlpHT);
  w.part[2] = c.take<float>(S * kMlpHid * kMlpHT);
  w.part[3] = c.take<float>(S * kMlpOutPad * kMlpHT);
  w.loss_part = c.take<float>(b / 64 + 1);
  if (bytes) *bytes = c.off + 256;
  return w;
}

// constant rows: ones after the inputs / activations, zeros beyond, zeroed dO
hipError_t init_train_ws(const TrainWs &w, int64_t B, hipStream_t st) {
  hipError_t e = launch_fill_u16(w.uT + kMlpIn * B, B, kBf16One, st);
  if (e == hipSuccess) e = launch_fill_u16(w.uT + (kMlpIn + 1) * B, (kMlpInPadT - kMlpIn - 1) * B, 0, st);
  for (int k = 0; k < 3 && e == hipSuccess; ++k) {
    e = launch_fill_u16(w.hT[k] + kMlpHid * B, B, kBf16One, st);
    if (e == hipSuccess) e = launch_fill_u16(w.hT[k] + (kMlpHid + 1) * B, (kMlpHT - kMlpHid - 1) * B, 0, st);
  }
  if (e == hipSuccess) e = launch_fill_u16(w.dO, kMlpInPad * B, 0, st);
  return e;
}

TrainArgs train_args(const TrainWs &w, const float *u, const float *r, int64_t n_pairs, int64_t B,
                     const double inv_scale[6]) {
  TrainArgs t{};
  t.u = u;
  t.r = r;
  t.n_pairs = n_pairs;
  t.perm_a = 1;
  t.perm_c = 0;
  t.row0 = 0;
  t.B = B;
  for (int k = 0; k < 6; ++k) t.inv_scale[k] = static_cast<float>(inv_scale[k]);
  t.uT = w.uT;
  for (int k = 0; k < 3; ++k) {
    t.aT[k] = w.aT[k];
    t.hT[k] = w.hT[k];
    t.dAT[k] = w.dAT[k];
  }
  t.dO = w.dO;
  t.dOT = w.dOT;
  t.loss_part = w.loss_part;
  return t;
}

WgradArgs wgrad_args(const TrainWs &w, int64_t B) {
  WgradArgs g{};
  g.job[0] = WgradJob{w.dAT[0], w.uT, w.part[0], 16, 1, 16};
  g.job[1] = WgradJob{w.dAT[1], w.hT[0], w.part[1], 16, 17, 16 * 17};
  g.job[2] = WgradJob{w.dAT[2], w.hT[1], w.part[2], 16, 17, 16 * 17};
  g.job[3] = WgradJob{w.dOT, w.hT[2], w.part[3], 1, 17, 17};
  g.tiles = 16 + 2 * 16 * 17 + 17;
  g.slices = w.slices;
  g.kslice = w.kslice;
  g.ld = B;
  return g;
}

// one batch: forward with saves, backward, weight-gradient partials
hipError_t batch_grad(const trk_mlp *m, const TrainArgs &t, const TrainWs &w, int x2, hipStream_t st) {
  const MlpDev d = dev_of(m);
  hipError_t e = launch_mlp_train_fwd(d, t, x2, st);
  if (e == hipSuccess) e = launch_mlp_train_bwd(d, t, st);
  if (e == hipSuccess) e = launch_mlp_wgrad(wgrad_args(w, t.B), st);
  return e;
}

uint64_t splitmix64(uint64_t &s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

}  // namespace

extern "C" int trk_mlp_create(const float *params_host, trk_mlp **out) {
  if (params_host == nullptr || out == nullptr) return fail(TRK_EINVAL, "params or out is NULL");
  trk_mlp *m = new (std::nothrow) trk_mlp;
  if (m == nullptr) return fail(TRK_ENOMEM, "host allocation");
  hipError_t e = hipMalloc(&m->w, 3 * kMlpNParam * sizeof(float));
  if (e == hipSuccess) e = hipMalloc(&m->bf, (kWfElems + kWbElems) * sizeof(uint16_t));
  if (e == hipSuccess) e = hipMalloc(&m->wi, kMlpInferElems * sizeof(uint16_t));
  if (e != hipSuccess) {
    (void)hipFree(m->w);
    (void)hipFree(m->bf);
    delete m;
    return fail(TRK_ENOMEM, std::string("network allocation: ") + hipGetErrorString(e));
  }
  m->m = m->w + kMlpNParam;
  m->v = m->m + kMlpNParam;
  m->w1f = m->bf;
  m->w2f = m->w1f + 256 * 32;
  m->w3f = m->w2f + 256 * 256;
  m->w4f = m->w3f + 256 * 256;
  m->w4b = m->w4f + 16 * 256;
  m->w3b = m->w4b + 256 * 32;
  m->w2b = m->w3b + 256 * 256;
  e = hipMemcpy(m->w, params_host, kMlpNParam * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(m->m, 0, 2 * kMlpNParam * sizeof(float));
  if (e == hipSuccess) e = hipMemset(m->bf, 0, (kWfElems + kWbElems) * sizeof(uint16_t));
  AdamArgs a = adam_base(m);
  a.mode = 3;
  if (e == hipSuccess) e = launch_mlp_adam(a, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    (void)hipFree(m->w);
    (void)hipFree(m->bf);
    (void)hipFree(m->wi);
    delete m;
    return hip_fail(e, "network upload");
  }
  *out = m;
  return TRK_OK;
}

extern "C" void trk_mlp_destroy(trk_mlp *m) {
  if (m == nullptr) return;
  (void)hipFree(m->w);
  (void)hipFree(m->bf);
  (void)hipFree(m->wi);
  delete m;
}

extern "C" int trk_mlp_get_params(const trk_mlp *m, float *params_host, void *stream) {
  if (m == nullptr || params_host == nullptr) return fail(TRK_EINVAL, "network or params is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(params_host, m->w, kMlpNParam * sizeof(float), hipMemcpyDeviceToHost, st),
          "parameter download");
  HIP_TRY(hipStreamSynchronize(st), "parameter download");
  return TRK_OK;
}

extern "C" int trk_mlp_forward(const trk_mlp *m, const float *u_dev, int64_t n, float *out_dev,
                               int32_t precision, void *stream) {
  if (m == nullptr) return fail(TRK_EINVAL, "network is NULL");
  if (n < 0) return fail(TRK_EINVAL, "n < 0");
  if (int r = check_prec(precision)) return r;
  if (n == 0) return TRK_OK;
  if (int r = check_dev(u_dev, "u")) return r;
  if (int r = check_dev(out_dev, "out")) return r;
  HIP_TRY(launch_mlp_forward(dev_of(m), u_dev, n, out_dev, precision == TRK_MLP_BF16X2,
                             static_cast<hipStream_t>(stream)),
          "network forward");
  return TRK_OK;
}

extern "C" size_t trk_mlp_workspace_size(int32_t batch) {
  if (batch <= 0) return 0;
  size_t b = 0;
  carve_train(nullptr, batch, &b);
  return b;
}

namespace {
int check_train_ws(void *ws, size_t bytes, int64_t B) {
  if (B <= 0 || B % 64 != 0) return fail(TRK_EINVAL, "batch rows must be a positive multiple of 64");
  const size_t need = trk_mlp_workspace_size(static_cast<int32_t>(B));
  if (bytes < need) return fail(TRK_ERANGE, "network workspace too small");
  return check_dev(ws, "workspace");
}
}  // namespace

extern "C" int trk_mlp_backward(const trk_mlp *m, const float *u_dev, const float *t_dev, int32_t n,
                                int32_t precision, float *grad_dev, float *loss_dev, void *workspace,
                                size_t workspace_bytes, void *stream) {
  if (m == nullptr) return fail(TRK_EINVAL, "network is NULL");
  if (int r = check_prec(precision)) return r;
  if (int r = check_train_ws(workspace, workspace_bytes, n)) return r;
  if (int r = check_dev(u_dev, "u")) return r;
  if (int r = check_dev(t_dev, "t")) return r;
  if (int r = check_dev(grad_dev, "grad")) return r;
  if (loss_dev != nullptr)
    if (int r = check_dev(loss_dev, "loss")) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const TrainWs w = carve_train(workspace, n, nullptr);
  const double one[6] = {1, 1, 1, 1, 1, 1};
  const TrainArgs t = train_args(w, u_dev, t_dev, n, n, one);
  HIP_TRY(init_train_ws(w, n, st), "workspace init");
  HIP_TRY(batch_grad(m, t, w, precision == TRK_MLP_BF16X2, st), "network backward");
  AdamArgs a = adam_base(const_cast<trk_mlp *>(m));
  a.mode = 2;
  a.slices = w.slices;
  for (int k = 0; k < 4; ++k) a.part[k] = w.part[k];
  a.grad_out = grad_dev;
  if (loss_dev != nullptr) {
    a.loss_part = w.loss_part;
    a.nloss = static_cast<int>(n / 64);
    a.loss_acc = loss_dev;
    a.loss_reset = 1;
    a.loss_scale = 1.0f / (6.0f * static_cast<float>(n));
  }
  HIP_TRY(launch_mlp_adam(a, st), "gradient reduction");
  return TRK_OK;
}

extern "C" int trk_mlp_adam_step(trk_mlp *m, const float *grad_dev, double lr, void *stream) {
  if (m == nullptr) return fail(TRK_EINVAL, "network is NULL");
  if (int r = check_dev(grad_dev, "grad")) return r;
  AdamArgs a = adam_base(m);
  a.mode = 1;
  a.grad_in = grad_dev;
  next_step(m, a, lr);
  HIP_TRY(launch_mlp_adam(a, static_cast<hipStream_t>(stream)), "Adam step");
  return TRK_OK;
}

extern "C" int trk_mlp_train(trk_mlp *m, const float *u_dev, const float *r_dev, int64_t n_pairs,
                             const double inv_scale[6], const trk_train_opts *o, float *loss_dev,
                             void *workspace, size_t workspace_bytes, void *stream) {
  if (m == nullptr || o == nullptr || inv_scale == nullptr)
    return fail(TRK_EINVAL, "network, options or scale is NULL");
  if (int r = check_prec(o->precision)) return r;
  if (o->epochs < 0) return fail(TRK_EINVAL, "epochs < 0");
  if (int r = check_train_ws(workspace, workspace_bytes, o->batch)) return r;
  if (n_pairs < o->batch || n_pairs > 0xffffffffLL)
    return fail(TRK_ERANGE, "n_pairs must lie in [batch, 2^32)");
  if (int r = check_dev(u_dev, "u")) return r;
  if (int r = check_dev(r_dev, "r")) return r;
  if (loss_dev != nullptr)
    if (int r = check_dev(loss_dev, "loss")) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t B = o->batch;
  const TrainWs w = carve_train(workspace, B, nullptr);
  HIP_TRY(init_train_ws(w, B, st), "workspace init");
  TrainArgs t = train_args(w, u_dev, r_dev, n_pairs, B, inv_scale);
  const int64_t spe = n_pairs / B;
  const int64_t total = spe * o->epochs;
  uint64_t rs = o->seed;
  const uint64_t n = static_cast<uint64_t>(n_pairs);
  const int x2 = o->precision == TRK_MLP_BF16X2;
  int64_t step = 0;
  for (int ep = 0; ep < o->epochs; ++ep) {
    uint64_t a = 1 + splitmix64(rs) % (n > 1 ? n - 1 : 1);
    while (std::gcd(a, n) != 1) a = a + 1 < n ? a + 1 : 1;
    t.perm_a = a;
    t.perm_c = splitmix64(rs) % n;
    for (int64_t k = 0; k < spe; ++k, ++step) {
      t.row0 = k * B;
      HIP_TRY(batch_grad(m, t, w, x2, st), "training step");
      AdamArgs ad = adam_base(m);
      ad.mode = 0;
      ad.slices = w.slices;
      for (int q = 0; q < 4; ++q) ad.part[q] = w.part[q];
      const double lr = o->lr_min + (o->lr0 - o->lr_min) * 0.5 *
                                        (1.0 + std::cos(kPi * static_cast<double>(step) /
                                                        static_cast<double>(total)));
      next_step(m, ad, lr);
      if (loss_dev != nullptr) {
        ad.loss_part = w.loss_part;
        ad.nloss = static_cast<int>(B / 64);
        ad.loss_acc = loss_dev + ep;
        ad.loss_reset = k == 0;
        ad.loss_scale = 1.0f / (6.0f * static_cast<float>(B) * static_cast<float>(spe));
      }
      HIP_TRY(launch_mlp_adam(ad, st), "Adam step");
    }
  }
  return TRK_OK;
}

// ------------------------------------------------------------------ section
struct trk_surrogate {
  const trk_lattice *sec = nullptr;
  trk_surrogate_opts o{};
  SurrDev c{};
  trk_surrogate_info info{};
};

namespace {

// Track the 13 central-difference probes through `lat` and return C, R.
int probe_map(const trk_lattice *lat, const double hw[6], double h_rel, void *buf, size_t ws_bytes,
              hipStream_t st, double C[6], double R[36]) {
  constexpr int kN = 13;
  double z[6][kN] = {};
  for (int k = 0; k < 6; ++k) {
    const double h = h_rel * hw[k];
    z[k][1 + 2 * k] = h;
    z[k][2 + 2 * k] = -h;
  }
  char *p = static_cast<char *>(buf);
  double *dz = reinterpret_cast<double *>(p);
  uint32_t *did = reinterpret_cast<uint32_t *>(p + 6 * kN * sizeof(double));
  int64_t *dlost = reinterpret_cast<int64_t *>(p + 1024);
  int64_t *dn = dlost + kN;
  void *ws = p + 4096;
  uint32_t ids[kN];
  int64_t lost[kN + 1];
  for (int i = 0; i < kN; ++i) {
    ids[i] = static_cast<uint32_t>(i);
    lost[i] = -1;
  }
  lost[kN] = kN;
  HIP_TRY(hipMemcpyAsync(dz, z, sizeof z, hipMemcpyHostToDevice, st), "probe upload");
  HIP_TRY(hipMemcpyAsync(did, ids, sizeof ids, hipMemcpyHostToDevice, st), "probe upload");
  HIP_TRY(hipMemcpyAsync(dlost, lost, sizeof lost, hipMemcpyHostToDevice, st), "probe upload");
  trk_beam b;
  b.x = dz;
  b.xp = dz + kN;
  b.y = dz + 2 * kN;
  b.yp = dz + 3 * kN;
  b.s = dz + 4 * kN;
  b.dp = dz + 5 * kN;
  b.id = did;
  b.lost_at = dlost;
  b.n_alive = dn;
  b.n_total = kN;
  trk_opts op{};
  op.p_ref_eV = 1e9;
  if (int r = trk_track(&b, lat, 1, &op, ws, ws_bytes, st)) return r;
  HIP_TRY(hipMemcpyAsync(z, dz, sizeof z, hipMemcpyDeviceToHost, st), "probe download");
  HIP_TRY(hipMemcpyAsync(ids, did, sizeof ids, hipMemcpyDeviceToHost, st), "probe download");
  HIP_TRY(hipMemcpyAsync(lost, dlost, sizeof lost, hipMemcpyDeviceToHost, st), "probe download");
  HIP_TRY(hipStreamSynchronize(st), "probe tracking");
  for (int i = 0; i < kN; ++i)
    if (lost[i] >= 0 || ids[i] != static_cast<uint32_t>(i))
      return fail(TRK_EINVAL, "a linear-map probe was lost in the section");
  for (int k = 0; k < 6; ++k) C[k] = z[k][0];
  for (int k = 0; k < 6; ++k) {
    const double h = h_rel * hw[k];
    for (int i = 0; i < 6; ++i) R[6 * i + k] = (z[i][1 + 2 * k] - z[i][2 + 2 * k]) / (2.0 * h);
  }
  return TRK_OK;
}

// periodic Courant--Snyder parameters and dispersion of block (i, i+1)
int twiss(const double R[36], int i, double &alpha, double &beta, double &gamma, double &eta,
          double &etap) {
  const double r00 = R[6 * i + i], r01 = R[6 * i + i + 1], r10 = R[6 * (i + 1) + i],
               r11 = R[6 * (i + 1) + i + 1];
  const double cmu = 0.5 * (r00 + r11);
  if (!(std::fabs(cmu) < 1.0)) return fail(TRK_EINVAL, "section linear map is not stable");
  double smu = std::sqrt(1.0 - cmu * cmu);
  if (r01 < 0.0) smu = -smu;
  beta = r01 / smu;
  alpha = (r00 - r11) / (2.0 * smu);
  gamma = -r10 / smu;
  const double det = (1.0 - r00) * (1.0 - r11) - r01 * r10;
  eta = ((1.0 - r11) * R[6 * i + 5] + r01 * R[6 * (i + 1) + 5]) / det;
  etap = (r10 * R[6 * i + 5] + (1.0 - r00) * R[6 * (i + 1) + 5]) / det;
  return TRK_OK;
}

}  // namespace

struct SurrWs {
  uint8_t *flags;
  int64_t *blk, *counts;
  uint32_t *adm, *rej;
  double *stage_z[6], *zin[6];
  uint32_t *stage_id;
  int64_t *stage_lost, *stage_n;
  double *sq_part, *sq;
  void *track_ws;
  size_t track_bytes;
};

namespace {

constexpr int64_t kSampleRound = int64_t(1) << 22;  // candidates per sampler round
constexpr int kSqBlocks = 1024;

size_t surr_ws_bytes(int64_t n_total, void *base, SurrWs *w) {
  const size_t n = static_cast<size_t>(std::max<int64_t>(n_total, 1));
  const size_t nb = static_cast<size_t>(nblocks(std::max<int64_t>(n_total, kSampleRound)));
  Carver c{static_cast<char *>(base)};
  SurrWs s;
  s.flags = c.take<uint8_t>(n);
  s.blk = c.take<int64_t>(2 * nb + 8);
  s.counts = c.take<int64_t>(8);
  s.adm = c.take<uint32_t>(n);
  s.rej = c.take<uint32_t>(n);
  for (int k = 0; k < 6; ++k) s.stage_z[k] = c.take<double>(n);
  for (int k = 0; k < 6; ++k) s.zin[k] = c.take<double>(n);
  s.stage_id = c.take<uint32_t>(n);
  s.stage_lost = c.take<int64_t>(n);
  s.stage_n = c.take<int64_t>(1);
  s.sq_part = c.take<double>(kSqBlocks * 8);
  s.sq = c.take<double>(8);
  s.track_bytes = workspace_bytes(n_total);
  s.track_ws = c.take<char>(s.track_bytes);
  if (w) *w = s;
  return c.off + 256;
}

BeamPtrs6 ptrs_of(const trk_beam *b) {
  BeamPtrs6 p;
  double *z[6];
  beam_ptrs(b, z);
  for (int k = 0; k < 6; ++k) p.z[k] = z[k];
  p.id = b->id;
  p.lost_at = b->lost_at;
  return p;
}

trk_beam stage_beam(const SurrWs &w, int64_t n_total) {
  trk_beam b;
  b.x = w.stage_z[0];
  b.xp = w.stage_z[1];
  b.y = w.stage_z[2];
  b.yp = w.stage_z[3];
  b.s = w.stage_z[4];
  b.dp = w.stage_z[5];
  b.id = w.stage_id;
  b.lost_at = w.stage_lost;
  b.n_alive = w.stage_n;
  b.n_total = n_total;
  return b;
}

int check_surr_ws(void *ws, size_t bytes, int64_t n_total) {
  const size_t need = surr_ws_bytes(n_total, nullptr, nullptr);
  if (bytes < need) return fail(TRK_ERANGE, "surrogate workspace too small");
  return check_dev(ws, "workspace");
}

}  // namespace

extern "C" int trk_surrogate_create(const trk_lattice *section, const trk_surrogate_opts *o,
                                    void *stream, trk_surrogate **out) {
  if (section == nullptr || o == nullptr || out == nullptr)
    return fail(TRK_EINVAL, "section, options or out is NULL");
  for (const trk_element &e : section->src)
    if (e.kind == TRK_RFCA || e.kind == TRK_WAKE || e.kind == TRK_RADKICK || e.kind == TRK_MAP2)
      return fail(TRK_EINVAL, "a surrogate section holds no RF, wake, random or explicit-map element");
  if (section->src.empty()) return fail(TRK_EINVAL, "empty section");
  for (int k = 0; k < 6; ++k)
    if (!(o->half_width[k] > 0.0)) return fail(TRK_EINVAL, "half widths must be > 0");
  if (!(o->margin >= 0.0 && o->margin < 1.0)) return fail(TRK_EINVAL, "margin must lie in [0, 1)");
  if (!(o->aper_a > 0.0 && o->aper_b > 0.0)) return fail(TRK_EINVAL, "aperture semi-axes must be > 0");
  const double h_rel = o->h_rel > 0.0 ? o->h_rel : 1e-4;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t tws = workspace_bytes(13);
  void *buf = nullptr;
  HIP_TRY(hipMalloc(&buf, 4096 + tws), "probe allocation");
  trk_surrogate *s = new (std::nothrow) trk_surrogate;
  if (s == nullptr) {
    (void)hipFree(buf);
    return fail(TRK_ENOMEM, "host allocation");
  }
  s->sec = section;
  s->o = *o;
  trk_surrogate_info &I = s->info;
  int r = probe_map(section, o->half_width, h_rel, buf, tws, st, I.C, I.R);
  // partial maps of every element prefix: largest beta and |eta| over the exits
  double ax = 0, bx = 0, gx = 0, eta = 0, etap = 0, ay = 0, by = 0, gy = 0, d1 = 0, d2 = 0;
  if (r == TRK_OK) r = twiss(I.R, 0, ax, bx, gx, eta, etap);
  if (r == TRK_OK) r = twiss(I.R, 2, ay, by, gy, d1, d2);
  double bhx = bx, bhy = by, eh = std::fabs(eta);
  const int ne = static_cast<int>(section->src.size());
  for (int k = 0; k < ne && r == TRK_OK; ++k) {
    trk_lattice *pl = nullptr;
    r = trk_lattice_create(section->src.data(), k + 1, &pl);
    double Cp[6], M[36];
    if (r == TRK_OK) r = probe_map(pl, o->half_width, h_rel, buf, tws, st, Cp, M);
    trk_lattice_destroy(pl);
    if (r != TRK_OK) break;
    const double p = M[0] * bx - M[1] * ax;
    bhx = std::max(bhx, (p * p + M[1] * M[1]) / bx);
    const double q = M[14] * by - M[15] * ay;
    bhy = std::max(bhy, (q * q + M[15] * M[15]) / by);
    eh = std::max(eh, std::fabs(M[0] * eta + M[1] * etap + M[5]));
  }
  (void)hipFree(buf);
  if (r != TRK_OK) {
    delete s;
    return r;
  }
  I.alpha_x = ax;
  I.beta_x = bx;
  I.gamma_x = gx;
  I.eta = eta;
  I.etap = etap;
  I.alpha_y = ay;
  I.beta_y = by;
  I.gamma_y = gy;
  I.beta_hat_x = bhx;
  I.beta_hat_y = bhy;
  I.eta_hat = eh;
  const double om = 1.0 - o->margin;
  I.lim = om * om;
  SurrDev &c = s->c;
  std::memcpy(c.C, I.C, sizeof c.C);
  std::memcpy(c.R, I.R, sizeof c.R);
  for (int k = 0; k < 6; ++k) {
    c.D[k] = 0.0;
    c.hw[k] = o->half_width[k];
  }
  c.gx = gx;
  c.ax2 = 2.0 * ax;
  c.bx = bx;
  c.gy = gy;
  c.ay2 = 2.0 * ay;
  c.by = by;
  c.eta = eta;
  c.etap = etap;
  c.bhx = bhx;
  c.bhy = bhy;
  c.eh = eh;
  c.inv_a = 1.0 / o->aper_a;
  c.inv_b = 1.0 / o->aper_b;
  c.lim = I.lim;
  // sampler box: the admitted set lies inside |x_beta| <= sqrt(J beta),
  // |x'_beta| <= sqrt(J gamma) with J <= a^2 lim / betahat, |delta| <= a sqrt(lim)/etahat
  const double pad = 1.0 + 1e-6;
  const double jxm = ((o->aper_a * o->aper_a) * I.lim) / bhx;
  const double jym = ((o->aper_b * o->aper_b) * I.lim) / bhy;
  const double dm = eh > 0.0 ? (o->aper_a * std::sqrt(I.lim)) / eh : o->half_width[5];
  double sw[6];
  sw[0] = (std::sqrt(jxm * bx) + std::fabs(eta) * dm) * pad;
  sw[1] = (std::sqrt(jxm * gx) + std::fabs(etap) * dm) * pad;
  sw[2] = std::sqrt(jym * by) * pad;
  sw[3] = std::sqrt(jym * gy) * pad;
  sw[4] = o->half_width[4];
  sw[5] = dm * pad;
  for (int k = 0; k < 6; ++k) {
    c.sw[k] = std::min(sw[k], o->half_width[k]);
    // the network sees the admitted set scaled into [-1, 1]
    c.inv_nw[k] = 1.0 / c.sw[k];
    I.sample_half_width[k] = c.sw[k];
    I.D[k] = 0.0;
  }
  *out = s;
  return TRK_OK;
}

extern "C" void trk_surrogate_destroy(trk_surrogate *s) { delete s; }

extern "C" int trk_surrogate_get_info(const trk_surrogate *s, trk_surrogate_info *out) {
  if (s == nullptr || out == nullptr) return fail(TRK_EINVAL, "surrogate or out is NULL");
  *out = s->info;
  return TRK_OK;
}

extern "C" size_t trk_surrogate_workspace_size(const trk_surrogate *s, int64_t n_total) {
  (void)s;
  return surr_ws_bytes(n_total, nullptr, nullptr);
}

extern "C" int trk_surrogate_gate(const trk_surrogate *s, const trk_beam *beam, uint8_t *admit_dev,
                                  void *stream) {
  if (s == nullptr) return fail(TRK_EINVAL, "surrogate is NULL");
  if (int r = check_beam(beam)) return r;
  if (beam->n_total == 0) return TRK_OK;
  if (int r = check_dev(admit_dev, "admit")) return r;
  HIP_TRY(launch_gate_flags(ptrs_of(beam), beam->n_alive, beam->n_total, s->c, admit_dev,
                            static_cast<hipStream_t>(stream)),
          "gate");
  return TRK_OK;
}

extern "C" int trk_surrogate_sample(const trk_surrogate *s, uint64_t seed, uint64_t first,
                                    trk_beam *beam, uint64_t *next_out, void *workspace,
                                    size_t workspace_bytes, void *stream) {
  if (s == nullptr || next_out == nullptr) return fail(TRK_EINVAL, "surrogate or next_out is NULL");
  if (int r = check_beam(beam)) return r;
  if (int r = check_surr_ws(workspace, workspace_bytes, beam->n_total)) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  SurrWs w;
  surr_ws_bytes(beam->n_total, workspace, &w);
  int64_t *base = w.counts + 3;
  HIP_TRY(launch_fill_u16(reinterpret_cast<uint16_t *>(base), 4, 0, st), "sampler init");
  const int64_t cap = beam->n_total;
  uint64_t c0 = first;
  int64_t got = 0;
  int idle = 0;
  while (got < cap) {
    HIP_TRY(launch_sample(s->c, seed, c0, kSampleRound, w.blk, ptrs_of(beam), base, cap, st), "sampler");
    c0 += static_cast<uint64_t>(kSampleRound);
    int64_t now = 0;
    HIP_TRY(hipMemcpyAsync(&now, base, sizeof now, hipMemcpyDeviceToHost, st), "sampler count");
    HIP_TRY(hipStreamSynchronize(st), "sampler count");
    idle = now == got ? idle + 1 : 0;
    if (idle >= 64) return fail(TRK_EINVAL, "the gate admits (almost) nothing of the sampler box");
    got = now;
  }
  HIP_TRY(hipMemcpyAsync(beam->n_alive, &cap, sizeof cap, hipMemcpyHostToDevice, st), "n_alive");
  HIP_TRY(hipStreamSynchronize(st), "n_alive");
  *next_out = c0;
  return TRK_OK;
}

extern "C" int trk_surrogate_pairs(const trk_surrogate *s, const trk_beam *beam, float *u_dev,
                                   float *r_dev, int64_t *n_pairs_dev, void *workspace,
                                   size_t workspace_bytes, void *stream) {
  if (s == nullptr) return fail(TRK_EINVAL, "surrogate is NULL");
  if (int r = check_beam(beam)) return r;
  if (int r = check_surr_ws(workspace, workspace_bytes, beam->n_total)) return r;
  if (int r = check_dev(u_dev, "u")) return r;
  if (int r = check_dev(r_dev, "r")) return r;
  if (int r = check_dev(n_pairs_dev, "n_pairs")) return r;
  if (beam->n_total == 0) return fail(TRK_EINVAL, "empty beam");
  hipStream_t st = static_cast<hipStream_t>(stream);
  SurrWs w;
  surr_ws_bytes(beam->n_total, workspace, &w);
  const BeamPtrs6 src = ptrs_of(beam);
  trk_beam sb = stage_beam(w, beam->n_total);
  const BeamPtrs6 stage = ptrs_of(&sb);
  HIP_TRY(launch_gate_split(src, beam->n_alive, beam->n_total, s->c, w.flags, w.blk, w.adm, w.rej,
                            w.counts, st),
          "gate");
  HIP_TRY(launch_gather(src, w.adm, w.counts, beam->n_total, stage, w.stage_n, w.zin, 0, st), "gather");
  trk_opts op{};
  op.p_ref_eV = 1e9;
  if (int r = trk_track(&sb, s->sec, 1, &op, w.track_ws, w.track_bytes, st)) return r;
  HIP_TRY(launch_pairs(stage, w.stage_n, beam->n_total, w.zin, s->c, u_dev, r_dev, n_pairs_dev, st),
          "pairs");
  return TRK_OK;
}

extern "C" int trk_surrogate_fit_scale(trk_surrogate *s, const float *r_dev, int64_t n,
                                       void *workspace, size_t workspace_bytes, void *stream) {
  if (s == nullptr) return fail(TRK_EINVAL, "surrogate is NULL");
  if (n <= 0) return fail(TRK_EINVAL, "no rows");
  if (int r = check_dev(r_dev, "r")) return r;
  if (int r = check_surr_ws(workspace, workspace_bytes, 1)) return r;
  hipStream_t st = static_cast<hipStream_t>(stream);
  SurrWs w;
  surr_ws_bytes(1, workspace, &w);
  const int nblk = static_cast<int>(std::min<int64_t>(kSqBlocks, nblocks(n)));
  HIP_TRY(launch_sumsq(r_dev, n, w.sq_part, nblk, w.sq, st), "scale reduction");
  double sq[8];
  HIP_TRY(hipMemcpyAsync(sq, w.sq, sizeof sq, hipMemcpyDeviceToHost, st), "scale download");
  HIP_TRY(hipStreamSynchronize(st), "scale reduction");
  for (int k = 0; k < 6; ++k) {
    const double d = k < kMlpDCol ? std::sqrt(sq[k] / static_cast<double>(n)) : 0.0;
    s->c.D[k] = d;
    s->info.D[k] = d;
  }
  return TRK_OK;
}

extern "C" int trk_surrogate_apply(const trk_surrogate *s, const trk_mlp *m, trk_beam *beam,
                                   int32_t first_pass, int32_t precision, int64_t *n_admitted_dev,
                                   void *workspace, size_t workspace_bytes, void *stream) {
  if (s == nullptr || m == nullptr) return fail(TRK_EINVAL, "surrogate or network is NULL");
  if (int r = check_prec(precision)) return r;
  if (int r = check_beam(beam)) return r;
  if (int r = check_surr_ws(workspace, workspace_bytes, beam->n_total)) return r;
  if (n_admitted_dev != nullptr)
    if (int r = check_dev(n_admitted_dev, "n_admitted")) return r;
  if (beam->n_total == 0) return TRK_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  SurrWs w;
  surr_ws_bytes(beam->n_total, workspace, &w);
  const BeamPtrs6 bp = ptrs_of(beam);
  trk_beam sb = stage_beam(w, beam->n_total);
  const BeamPtrs6 stage = ptrs_of(&sb);
  HIP_TRY(launch_gate_split(bp, beam->n_alive, beam->n_total, s->c, w.flags, w.blk, w.adm, w.rej,
                            w.counts, st),
          "gate");
  // fallback: the rejected particles through the section element by element,
  // left in gather order (their losses marked, not compacted), so the
  // scatter back writes the beam in index order; the whole beam is compacted
  // once at the end
  HIP_TRY(launch_gather(bp, w.rej, w.counts + 1, beam->n_total, stage, w.stage_n, nullptr, 1, st),
          "gather");
  trk_opts op{};
  op.p_ref_eV = 1e9;
  op.first_pass = first_pass;
  if (int r = track_impl(&sb, s->sec, 1, &op, w.track_ws, w.track_bytes, st, false)) return r;
  const MlpDev md = dev_of(m);
  HIP_TRY(profiled_call(1, st,
                        [&] {
                          return launch_surr_infer(md, s->c, bp, w.adm, w.counts, beam->n_total,
                                                   precision == TRK_MLP_BF16X2, st);
                        }),
          "surrogate inference");
  HIP_TRY(launch_scatter_back(stage, w.counts + 1, beam->n_total, bp, st), "scatter");
  if (n_admitted_dev != nullptr)
    HIP_TRY(hipMemcpyAsync(n_admitted_dev, w.counts, sizeof(int64_t), hipMemcpyDeviceToDevice, st),
            "admitted count");
  return trk_compact_lost(beam, w.track_ws, w.track_bytes, st);
}
