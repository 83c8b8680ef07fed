// mlp.h -- device records and launchers of the learned section surrogate
// (the residual network in mlp.hip, the gate, sampler and section
// replacement in surr.hip).
#pragma once
#include "trk_internal.h"

namespace trk {

constexpr int kMlpIn = TRK_MLP_IN, kMlpHid = TRK_MLP_HID, kMlpOut = TRK_MLP_OUT;
constexpr int kMlpSCol = 4;      // s: not a network input
constexpr int kMlpDCol = 5;      // delta: unchanged by the section
constexpr int kMlpInPad = 32;    // K of layer 1; row length of dO and of the W1, W4^T copies
constexpr int kMlpInPadT = 16;   // rows of u^T: 6 inputs, a row of ones, zeros
constexpr int kMlpOutPad = 16;   // rows of the W4 copy and of dO^T
constexpr int kMlpHT = 272;      // rows of h^T: 256 activations, a row of ones, zeros
constexpr int kMlpInK = 16;      // K of layer 1 in inference (6 inputs, zero-padded)
// inference weight copies (one allocation): W1 [256][16], W2 and W3 [256][256]
// and W4 [32][256] (6 rows used) with input columns in tile position order
constexpr int64_t kOffW2i = 256 * kMlpInK;
constexpr int64_t kOffW3i = kOffW2i + 256 * 256;
constexpr int64_t kOffW4i = kOffW3i + 256 * 256;
constexpr int64_t kMlpInferElems = kOffW4i + 32 * 256;
constexpr int64_t kOffW1 = 0;
constexpr int64_t kOffB1 = kOffW1 + kMlpHid * kMlpIn;
constexpr int64_t kOffW2 = kOffB1 + kMlpHid;
constexpr int64_t kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int64_t kOffW3 = kOffB2 + kMlpHid;
constexpr int64_t kOffB3 = kOffW3 + kMlpHid * kMlpHid;
constexpr int64_t kOffW4 = kOffB3 + kMlpHid;
constexpr int64_t kOffB4 = kOffW4 + kMlpOut * kMlpHid;
constexpr int64_t kMlpNParam = kOffB4 + kMlpOut;
static_assert(kMlpNParam == TRK_MLP_NPARAM, "parameter count");

// bf16 weight copies (forward: [out][in], backward: [in][out]) and FP32 biases
struct MlpDev {
  const uint16_t *w1f;  // [256][32]
  const uint16_t *w2f;  // [256][256]
  const uint16_t *w3f;  // [256][256]
  const uint16_t *w4f;  // [16][256]
  const uint16_t *w4b;  // [256][32]
  const uint16_t *w3b;  // [256][256]
  const uint16_t *w2b;  // [256][256]
  const float *b1, *b2, *b3, *b4;
  uint16_t *wi;         // [kMlpInferElems] inference copies (written per inference call)
};

struct TrainArgs {
  const float *u, *r;      // pairs [n_pairs][8]
  int64_t n_pairs;
  uint64_t perm_a, perm_c; // batch row g reads pair (perm_a g + perm_c) mod n_pairs
  int64_t row0;            // first row of this step within the epoch
  int64_t B;               // batch rows (multiple of 64)
  float inv_scale[6];      // target t_k = r_k inv_scale_k
  uint16_t *uT;            // [16][B]
  float *aT[3];            // [256][B] pre-activations
  uint16_t *hT[3];         // [272][B] activations (hi part), ones row at 256
  uint16_t *dO;            // [B][32]
  uint16_t *dOT;           // [16][B]
  uint16_t *dAT[3];        // [256][B]
  float *loss_part;        // [B/64] squared-error sums of the tiles
};

struct WgradJob {
  const uint16_t *a, *b;   // [16 mt][ld], [16 nt][ld]
  float *out;              // [slices][16 mt][16 nt]
  int mt, nt, ntiles;
};
struct WgradArgs {
  WgradJob job[4];
  int tiles, slices;
  int64_t kslice, ld;
};

struct AdamArgs {
  int mode;                // 0 partials + Adam, 1 given gradient + Adam, 2 partials -> grad_out, 3 copies only
  int slices;
  float *w, *m, *v;        // master FP32 state
  const float *grad_in;
  float *grad_out;
  const float *part[4];    // split-K partials of the four layers
  double lr, b1, b2, omb1, omb2, bc1, bc2, eps;
  uint16_t *w1f, *w2f, *w3f, *w4f, *w4b, *w3b, *w2b;
  const float *loss_part;  // or null: per-tile squared-error sums
  int nloss;
  int loss_reset;          // 1: *loss_acc = sum * loss_scale, else +=
  float loss_scale;
  float *loss_acc;
};

hipError_t launch_mlp_forward(const MlpDev &m, const float *u, int64_t n, float *out, int x2,
                              hipStream_t st);
hipError_t launch_mlp_train_fwd(const MlpDev &m, const TrainArgs &t, int x2, hipStream_t st);
hipError_t launch_mlp_train_bwd(const MlpDev &m, const TrainArgs &t, hipStream_t st);
hipError_t launch_mlp_wgrad(const WgradArgs &w, hipStream_t st);
hipError_t launch_mlp_adam(const AdamArgs &a, hipStream_t st);
hipError_t launch_fill_u16(uint16_t *p, int64_t n, uint16_t v, hipStream_t st);

// ---------------------------------------------------------------- surrogate
// Section constants (host-computed, passed by value).
struct SurrDev {
  double C[6], R[36], D[6];
  double hw[6], inv_nw[6], sw[6];  // inv_nw = 1/sw: network input scale
  double gx, ax2, bx, gy, ay2, by, eta, etap, bhx, bhy, eh, inv_a, inv_b, lim;
};

struct BeamPtrs6 {
  double *z[6];
  uint32_t *id;
  int64_t *lost_at;
};

// stable split of the alive particles [0, *n_alive) into admitted and
// rejected index lists; counts[0] = admitted, counts[1] = rejected
hipError_t launch_gate_split(const BeamPtrs6 &b, const int64_t *n_alive, int64_t n_total,
                             const SurrDev &c, uint8_t *flags, int64_t *blk, uint32_t *adm,
                             uint32_t *rej, int64_t *counts, hipStream_t st);
// flags only (0/1 per particle, 0 beyond *n_alive)
hipError_t launch_gate_flags(const BeamPtrs6 &b, const int64_t *n_alive, int64_t n_total,
                             const SurrDev &c, uint8_t *flags, hipStream_t st);
// dst[j] = src[list[j]] for j < *count; dst ids = j (mode 0) or list[j] (mode 1);
// zin (optional) receives a copy of the coordinates; *dst_n = *count
hipError_t launch_gather(const BeamPtrs6 &src, const uint32_t *list, const int64_t *count,
                         int64_t n_total, const BeamPtrs6 &dst, int64_t *dst_n, double *const *zin,
                         int id_mode, hipStream_t st);
// beam[stage.id[j]] = stage[j] (coordinates and lost_at) for j < *count
hipError_t launch_scatter_back(const BeamPtrs6 &stage, const int64_t *count, int64_t n_total,
                               const BeamPtrs6 &beam, hipStream_t st);
// training pairs from the tracked stage (survivors j < *n_stage, ids = input slots)
hipError_t launch_pairs(const BeamPtrs6 &stage, const int64_t *n_stage, int64_t n_total,
                        double *const *zin, const SurrDev &c, float *u, float *r, int64_t *n_pairs,
                        hipStream_t st);
// sum over rows of r[k]^2 -> sumsq[8] (fixed-order, two kernels)
hipError_t launch_sumsq(const float *r, int64_t n, double *part, int nblk, double *sumsq,
                        hipStream_t st);
// network + linear part on the admitted list, written back into the beam
hipError_t launch_surr_infer(const MlpDev &m, const SurrDev &c, const BeamPtrs6 &b,
                             const uint32_t *adm, const int64_t *n_adm, int64_t n_total, int x2,
                             hipStream_t st);
// candidates c0 .. c0+M-1 of the sampler: admitted ones appended at
// out[*base + rank] while below cap; *base advanced by the admitted count
hipError_t launch_sample(const SurrDev &c, uint64_t seed, uint64_t c0, int64_t M, int64_t *blk,
                         const BeamPtrs6 &out, int64_t *base, int64_t cap, hipStream_t st);

}  // namespace trk
