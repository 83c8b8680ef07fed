"""CPU oracle of the learned section surrogate (plain numpy, FP64).

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It shares no code
with the HIP path.

The surrogate replaces a fixed lattice section (the first ten cells of the
storage ring) by

    y = C + R z + D * MLP(N(z)),

where C = map(0) and R = the Jacobian of the section map at the origin (the
linear transfer matrix of the paper's first-order tracking), N scales each
input coordinate by the half width of the training box, D is the
per-coordinate RMS of the residual y - (C + R z) over the training pairs, and
MLP is a residual network 6 -> 256 -> 256 -> 256 -> 6 with SiLU activations
and skip connections around the two hidden 256 -> 256 layers.  The network
weights that enter the matrix products are bfloat16 (rounded to nearest even
from FP32 master weights); biases stay FP32.  Particles outside the training
box or above a linear Courant--Snyder amplitude bound are not admitted and are
tracked through the section element by element.

What is computed here, in the order the functions follow:

* ``bf16_rne``      rounding of binary32 to bfloat16 (8-bit significand),
                    round to nearest, ties to even;
* ``linear_map``    C and R by central differences of the oracle tracker;
* ``twiss``         periodic Courant--Snyder parameters and dispersion of a
                    2x2 (plus dispersion column) block of R;
* ``gate_constants``/``gate``  the admission test;
* ``forward`` / ``loss_and_grad``  the network and its exact gradient;
* ``loss_and_grad_bf16``  the gradient with the bfloat16 rounding points of
                    a matrix-core training step;
* ``adam``          one Adam step (Kingma & Ba, ICLR 2015, Algorithm 1) in
                    FP64 arithmetic on FP32-stored state.
"""
from __future__ import annotations

import math
from typing import Dict, Sequence, Tuple

import numpy as np

N_IN, N_HID, N_OUT = 6, 256, 6
# parameter vector layout (FP32 master copy)
SHAPES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)),
          ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_HID)), ("b3", (N_HID,)),
          ("W4", (N_OUT, N_HID)), ("b4", (N_OUT,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)   # 134918
S_COORD = 4        # s (path-length deviation): not a network input
D_COORD = 5        # delta: passes through the section unchanged


def unpack(p: np.ndarray) -> Dict[str, np.ndarray]:
    """Views of the parameter vector by name."""
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = p[o:o + n].reshape(shp)
        o += n
    return out


def init_params(seed: int) -> np.ndarray:
    """The seeded initial parameters (a shared input, not arithmetic of the
    method): see paper_1710_07350_amd.inputs.mlp_init_params."""
    from paper_1710_07350_amd import inputs
    return inputs.mlp_init_params(seed)


# ---------------------------------------------------------------- bfloat16
def bf16_rne(x) -> np.ndarray:
    """Round binary32 values to the nearest bfloat16 (ties to even), returned
    as binary32.  bfloat16 keeps the sign, the 8 exponent bits and the top 7
    fraction bits of binary32; the discarded 16 bits decide the rounding.
    (Finite inputs only.)"""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    low = b & 0xFFFF
    keep = b >> 16
    up = (low > 0x8000) | ((low == 0x8000) & ((keep & 1) == 1))
    keep = keep + up.astype(np.uint64)
    return (keep << 16).astype(np.uint32).view(np.float32)


def split_bf16x2(x32: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """x ~ hi + lo with hi = bf16(x) and lo = bf16(x - hi) (the difference
    is exact in binary32)."""
    x32 = np.asarray(x32, dtype=np.float32)
    hi = bf16_rne(x32)
    lo = bf16_rne(x32 - hi)
    return hi, lo


def _mfma_input(h64: np.ndarray, mode: str) -> np.ndarray:
    """Value of an activation as it enters a matrix product."""
    if mode == "exact":
        return h64
    h32 = h64.astype(np.float32)
    if mode == "bf16":
        return bf16_rne(h32).astype(np.float64)
    hi, lo = split_bf16x2(h32)
    return hi.astype(np.float64) + lo.astype(np.float64)


def silu(a):
    return a / (1.0 + np.exp(-a))


def dsilu(a):
    s = 1.0 / (1.0 + np.exp(-a))
    return s * (1.0 + a * (1.0 - s))


def weights(p: np.ndarray, round_weights: bool = True) -> Dict[str, np.ndarray]:
    """FP64 copies of the parameters; the matrices rounded to bfloat16 when
    ``round_weights`` (the network as the kernels evaluate it)."""
    P = unpack(np.asarray(p))
    out = {}
    for name, arr in P.items():
        if name.startswith("W") and round_weights:
            out[name] = bf16_rne(arr.astype(np.float32)).astype(np.float64)
        else:
            out[name] = np.asarray(arr, dtype=np.float64)
    return out


def forward(p, u, mode: str = "exact", round_weights: bool = True, cache: bool = False):
    """Network output o[n][6] for normalised inputs u[n][6] (FP64).

    mode: "exact" (activations in FP64), "bf16" (every activation rounded to
    bfloat16 where it enters a product) or "bf16x2" (entered as the sum of two
    bfloat16 numbers)."""
    W = weights(p, round_weights)
    u = np.asarray(u, dtype=np.float64).copy()
    u[:, S_COORD] = 0.0
    a1 = _mfma_input(u, mode) @ W["W1"].T + W["b1"]
    h1 = silu(a1)
    a2 = _mfma_input(h1, mode) @ W["W2"].T + W["b2"]
    h2 = h1 + silu(a2)
    a3 = _mfma_input(h2, mode) @ W["W3"].T + W["b3"]
    h3 = h2 + silu(a3)
    o = _mfma_input(h3, mode) @ W["W4"].T + W["b4"]
    if cache:
        return o, dict(u=u, a1=a1, h1=h1, a2=a2, h2=h2, a3=a3, h3=h3, W=W)
    return o


def loss_and_grad(p, u, t, round_weights: bool = True):
    """Mean-square loss L = (1/(6n)) sum_b sum_k (o_bk - t_bk)^2 and its
    exact gradient with respect to the parameters (FP64, activations exact;
    the bfloat16 rounding of weights is passed straight through)."""
    o, c = forward(p, u, "exact", round_weights, cache=True)
    n = o.shape[0]
    W = c["W"]
    d = o - t
    loss = float((d * d).sum() / (6.0 * n))
    dO = d * (2.0 / (6.0 * n))
    g = {}
    g["W4"] = dO.T @ c["h3"]
    g["b4"] = dO.sum(0)
    dh3 = dO @ W["W4"]
    dA3 = dh3 * dsilu(c["a3"])
    g["W3"] = dA3.T @ c["h2"]
    g["b3"] = dA3.sum(0)
    dh2 = dh3 + dA3 @ W["W3"]
    dA2 = dh2 * dsilu(c["a2"])
    g["W2"] = dA2.T @ c["h1"]
    g["b2"] = dA2.sum(0)
    dh1 = dh2 + dA2 @ W["W2"]
    dA1 = dh1 * dsilu(c["a1"])
    g["W1"] = dA1.T @ c["u"]
    g["b1"] = dA1.sum(0)
    flat = np.concatenate([g[name].reshape(-1) for name, _ in SHAPES])
    return loss, flat


def loss_and_grad_bf16(p, u, t, mode: str = "bf16x2"):
    """Loss and gradient with the rounding points of a bfloat16 matrix-core
    training step, FP64 arithmetic everywhere else:

      forward in `mode` (activations entering products as bfloat16 or as the
      sum of two), output error dO = bf16((o - t) 2/(6n)) with 2/(6n) taken
      in binary32;
      dh3 = dO W4;  dA_l = bf16(dh_l silu'(a_l));  dh_{l-1} = dh_l + dA_l W_l;
      weight gradients dA_l^T bf16(h_{l-1}) (layer 1: bf16(u)), bias
      gradients sum_rows dA_l, output layer dO^T bf16(h3) and sum_rows dO.

    Returns (loss, flat gradient, parts) where parts holds the rounded
    operands and the values before rounding (for error bounds)."""
    o, c = forward(p, u, mode, True, cache=True)
    W = c["W"]
    n = o.shape[0]
    scale = float(np.float32(2.0) / np.float32(6.0 * n))
    d = o - t
    loss = float((d * d).sum() / (6.0 * n))
    pre = {"dO": d * scale}
    rnd = {"dO": bf16_rne(pre["dO"].astype(np.float32)).astype(np.float64)}
    dh = {3: rnd["dO"] @ W["W4"]}
    for layer, wname in ((3, "W3"), (2, "W2"), (1, None)):
        key = f"dA{layer}"
        pre[key] = dh[layer] * dsilu(c[f"a{layer}"])
        rnd[key] = bf16_rne(pre[key].astype(np.float32)).astype(np.float64)
        if wname is not None:
            dh[layer - 1] = dh[layer] + rnd[key] @ W[wname]
    for name, src in (("u", c["u"]), ("h1", c["h1"]), ("h2", c["h2"]), ("h3", c["h3"])):
        pre[name] = src
        rnd[name] = bf16_rne(src.astype(np.float32)).astype(np.float64)
    g = {"W4": rnd["dO"].T @ rnd["h3"], "b4": rnd["dO"].sum(0),
         "W3": rnd["dA3"].T @ rnd["h2"], "b3": rnd["dA3"].sum(0),
         "W2": rnd["dA2"].T @ rnd["h1"], "b2": rnd["dA2"].sum(0),
         "W1": rnd["dA1"].T @ rnd["u"], "b1": rnd["dA1"].sum(0)}
    flat = np.concatenate([g[name].reshape(-1) for name, _ in SHAPES])
    parts = dict(pre=pre, rnd=rnd, dh=dh, o=o, cache=c)
    return loss, flat, parts


# ---------------------------------------------------------------- Adam
def adam(w32, m32, v32, g32, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step on FP32-stored state, evaluated in FP64.

        m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2
        w <- w - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

    b^t is the product of t factors b (t = step >= 1), multiplied in order."""
    p1 = 1.0
    p2 = 1.0
    for _ in range(step):
        p1 = p1 * b1
        p2 = p2 * b2
    bc1 = 1.0 - p1
    bc2 = 1.0 - p2
    omb1 = 1.0 - b1
    omb2 = 1.0 - b2
    g = np.asarray(g32, dtype=np.float32).astype(np.float64)
    m = b1 * np.asarray(m32, np.float32).astype(np.float64) + omb1 * g
    v = b2 * np.asarray(v32, np.float32).astype(np.float64) + omb2 * (g * g)
    upd = (lr * (m / bc1)) / (np.sqrt(v / bc2) + eps)
    w = np.asarray(w32, np.float32).astype(np.float64) - upd
    return w.astype(np.float32), m.astype(np.float32), v.astype(np.float32)


# ---------------------------------------------------------------- linear map
def probe_points(hw: Sequence[float], h_rel: float) -> np.ndarray:
    """13 probe particles: the origin, then +h and -h along each coordinate,
    h_k = h_rel * hw_k."""
    Z = np.zeros((6, 13))
    for k in range(6):
        h = h_rel * hw[k]
        Z[k, 1 + 2 * k] = h
        Z[k, 2 + 2 * k] = -h
    return Z


def fd_map(out: np.ndarray, hw: Sequence[float], h_rel: float):
    """C and R from the tracked probes: C = out(0), column k of R =
    (out(+h e_k) - out(-h e_k)) / (2 h)."""
    C = out[:, 0].copy()
    R = np.zeros((6, 6))
    for k in range(6):
        h = h_rel * hw[k]
        R[:, k] = (out[:, 1 + 2 * k] - out[:, 2 + 2 * k]) / (2.0 * h)
    return C, R


def linear_map(orc, lattice, hw, h_rel: float):
    """Track the probes through `lattice` with the oracle tracker (one pass,
    ids 0..12, so the compaction leaves them in order)."""
    Z = probe_points(hw, h_rel)
    b = orc.Beam(Z, np.arange(13, dtype=np.uint32), np.full(13, -1, np.int64))
    orc.track(b, lattice, 1)
    assert (b.lost_at < 0).all()
    return fd_map(b.z, hw, h_rel)


# ---------------------------------------------------------------- gate
def twiss(R, i: int):
    """Periodic Courant--Snyder parameters of the 2x2 block (i, i+1) of R:
    cos mu = (R00 + R11)/2, sin mu with the sign of R01, beta = R01/sin mu,
    alpha = (R00 - R11)/(2 sin mu), gamma = -R10/sin mu; and the periodic
    dispersion (eta, eta') solving (I - R2) (eta, eta') = (R05, R15)."""
    r00, r01, r10, r11 = R[i, i], R[i, i + 1], R[i + 1, i], R[i + 1, i + 1]
    cmu = 0.5 * (r00 + r11)
    if not abs(cmu) < 1.0:
        raise ValueError("section linear map is not stable in this plane")
    smu = math.sqrt(1.0 - cmu * cmu)
    if r01 < 0.0:
        smu = -smu
    beta = r01 / smu
    alpha = (r00 - r11) / (2.0 * smu)
    gamma = -r10 / smu
    det = (1.0 - r00) * (1.0 - r11) - r01 * r10
    eta = ((1.0 - r11) * R[i, 5] + r01 * R[i + 1, 5]) / det
    etap = (r10 * R[i, 5] + (1.0 - r00) * R[i + 1, 5]) / det
    return alpha, beta, gamma, eta, etap


def gate_constants(R_sec, partial_maps, hw, margin: float, a: float, b: float):
    """Constants of the admission test: periodic Twiss of the section map,
    the largest beta (x, y) and |eta| over the entrance and the exits of the
    elements whose partial maps (entrance to element exit) are given."""
    ax, bx, gx, eta, etap = twiss(R_sec, 0)
    ay, by, gy, _, _ = twiss(R_sec, 2)
    bhx, bhy, eh = bx, by, abs(eta)
    for M in partial_maps:
        p = M[0, 0] * bx - M[0, 1] * ax
        bhx = max(bhx, (p * p + M[0, 1] * M[0, 1]) / bx)
        q = M[2, 2] * by - M[2, 3] * ay
        bhy = max(bhy, (q * q + M[2, 3] * M[2, 3]) / by)
        eh = max(eh, abs(M[0, 0] * eta + M[0, 1] * etap + M[0, 5]))
    om = 1.0 - margin
    return dict(gx=gx, ax2=2.0 * ax, bx=bx, gy=gy, ay2=2.0 * ay, by=by, eta=eta, etap=etap,
                bhx=bhx, bhy=bhy, eh=eh, inv_a=1.0 / a, inv_b=1.0 / b, lim=om * om,
                hw=tuple(float(h) for h in hw))


def gate(z: np.ndarray, g: dict) -> np.ndarray:
    """Admission test per particle (z[6][n], FP64; each operation separate):
    inside the box |z_k| <= hw_k for k != s, and the linear amplitude bound
    (xhat/a)^2 + (yhat/b)^2 <= (1 - margin)^2 with
    xhat = sqrt(J_x betahat_x) + etahat |delta|, yhat = sqrt(J_y betahat_y),
    J = gamma u^2 + 2 alpha u u' + beta u'^2 of the betatron part
    (u = x - eta delta, u' = x' - eta' delta)."""
    x, xp, y, yp, s, d = z
    hw = g["hw"]
    box = np.ones(z.shape[1], dtype=bool)
    for k in (0, 1, 2, 3, 5):
        box &= np.abs(z[k]) <= hw[k]
    xb = x - g["eta"] * d
    xpb = xp - g["etap"] * d
    jx = ((g["gx"] * xb) * xb + (g["ax2"] * xb) * xpb) + (g["bx"] * xpb) * xpb
    jy = ((g["gy"] * y) * y + (g["ay2"] * y) * yp) + (g["by"] * yp) * yp
    with np.errstate(invalid="ignore"):
        xh = np.sqrt(np.maximum(jx * g["bhx"], 0.0)) + g["eh"] * np.abs(d)
        yh = np.sqrt(np.maximum(jy * g["bhy"], 0.0))
    ux = xh * g["inv_a"]
    uy = yh * g["inv_b"]
    q = ux * ux + uy * uy
    return box & (q <= g["lim"])


def sample_widths(g: dict, a: float, b: float) -> np.ndarray:
    """Half widths of the sampler's box, which contains every admitted point:
    J_x <= a^2 lim / betahat_x, J_y <= b^2 lim / betahat_y and
    |delta| <= a sqrt(lim) / etahat bound |x| <= sqrt(J_x beta_x) + |eta||delta|,
    |x'| <= sqrt(J_x gamma_x) + |eta'||delta|, |y| <= sqrt(J_y beta_y),
    |y'| <= sqrt(J_y gamma_y); each widened by 1e-6 relative and capped by the
    training box."""
    hw = g["hw"]
    pad = 1.0 + 1e-6
    lim = g["lim"]
    jxm = ((a * a) * lim) / g["bhx"]
    jym = ((b * b) * lim) / g["bhy"]
    dm = (a * math.sqrt(lim)) / g["eh"] if g["eh"] > 0.0 else hw[5]
    sw = [(math.sqrt(jxm * g["bx"]) + abs(g["eta"]) * dm) * pad,
          (math.sqrt(jxm * g["gx"]) + abs(g["etap"]) * dm) * pad,
          math.sqrt(jym * g["by"]) * pad,
          math.sqrt(jym * g["gy"]) * pad,
          hw[4],
          dm * pad]
    return np.array([min(sw[k], hw[k]) for k in range(6)])


TAG_SAMPLE = 5


def draw(orc, sw, seed: int, cand: int) -> np.ndarray:
    """Candidate `cand` of the sampler: words of Philox4x32-10 at counters
    (cand_lo, cand_hi, 5, 0) and (.., 1), key (seed_lo, seed_hi);
    z_k = (2 u_k - 1) sw_k with u_k = (w_k + 1/2) 2^-32."""
    key = (seed & 0xFFFFFFFF, seed >> 32)
    lo, hi = cand & 0xFFFFFFFF, cand >> 32
    w = orc.philox4x32_10((lo, hi, TAG_SAMPLE, 0), key) + orc.philox4x32_10((lo, hi, TAG_SAMPLE, 1), key)
    z = np.empty(6)
    for k in range(6):
        u = (float(w[k]) + 0.5) * 2.0 ** -32
        z[k] = (2.0 * u - 1.0) * sw[k]
    return z


def sample(orc, g: dict, sw, seed: int, first: int, n: int) -> Tuple[np.ndarray, int]:
    """The first n admitted candidates from `first` on, in candidate order;
    returns z[6][n] and the index of the last candidate examined plus one."""
    out = []
    c = first
    while len(out) < n:
        z = draw(orc, sw, seed, c)
        if _gate_one(z, g):
            out.append(z)
        c += 1
    return np.array(out).T, c


def _gate_one(z, g) -> bool:
    return bool(gate(np.asarray(z, dtype=np.float64).reshape(6, 1), g)[0])


# ---------------------------------------------------------------- surrogate
def normalise(z: np.ndarray, hw) -> np.ndarray:
    """u[n][6] = z_k / hw_k (s set to 0)."""
    u = np.empty((z.shape[1], 6))
    for k in range(6):
        u[:, k] = z[k] * (1.0 / hw[k])
    u[:, S_COORD] = 0.0
    return u


def linear_part(C, R, z: np.ndarray) -> np.ndarray:
    """C + R z evaluated per output as ((C_i + R_i0 z_0) + R_i1 z_1) + ...,
    skipping exactly-zero coefficients."""
    out = np.empty_like(z)
    for i in range(6):
        acc = np.full(z.shape[1], C[i])
        for j in range(6):
            if R[i, j] != 0.0:
                acc = acc + R[i, j] * z[j]
        out[i] = acc
    return out


def residual(C, R, z_in, z_out) -> np.ndarray:
    """Training residual r = y - (C + R z) as FP32 [n][6] (delta row 0)."""
    r = (z_out - linear_part(C, R, z_in)).astype(np.float32)
    r[D_COORD] = 0.0
    return np.ascontiguousarray(r.T)


def apply(p, C, R, D, hw, z, mode: str = "bf16x2") -> np.ndarray:
    """Surrogate output y = C + R z + D o for admitted particles z[6][n]."""
    o = forward(p, normalise(z, hw).astype(np.float32).astype(np.float64), mode)
    y = linear_part(C, R, z)
    for i in range(5):
        y[i] = y[i] + D[i] * o[:, i]
    y[D_COORD] = z[D_COORD]
    return y
