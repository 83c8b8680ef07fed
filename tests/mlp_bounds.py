"""Element-wise error bounds of the network's matrix-core evaluation against
the oracle's FP64 evaluation with the same bfloat16 rounding points.

Model of the device arithmetic (binary32 unit roundoff u = 2^-24):
* a matrix-core product of K bfloat16 pairs accumulated in binary32 differs
  from the exact sum by at most gamma_K u sum |a||b|, gamma_K = K u/(1 - K u)
  (any summation order with one rounding per addition);
* each other binary32 operation rounds once (relative u);
* the device SiLU, a * rcp(1 + exp2(-a log2 e)), has relative error at most
  (|a| + 8) u (the exponent's argument error is amplified by |a|; exp2 and
  the reciprocal are within one ulp); its derivative
  s (1 + a (1 - s)) absolute error at most 2 (|a| + 4)^2 u;
* |silu'| <= 1.1 and |silu''| <= 0.5 everywhere;
* an activation entering a product as hi + lo = bf16(h) + bf16(h - hi) is
  within 2^-18 |h| of h; the skip path of the inference kernel reads the
  previous activation back as hi + lo;
* a value rounded to one bfloat16 gives the same result on both sides unless
  the two unrounded values lie on opposite sides of a rounding midpoint: where
  the oracle's value lies within the deviation bound of a midpoint, the
  rounded operand may differ by one bfloat16 ulp.

Two forms of every bound: the worst case (lam = None: gamma_K, and deviations
propagated through sum_k |W_jk| dx_k), and the probabilistic one of Higham and
Mary ("A new approach to probabilistic rounding error analysis", SIAM J. Sci.
Comput. 41, 2019): with rounding errors independent and of mean zero, a sum of
K products is within gamma~_K(lam) sum |a||b|, gamma~_K(lam) =
exp(lam sqrt(K) u + K u^2/(1 - u)) - 1, with probability at least
1 - 2K exp(-lam^2 (1-u)^2 / 2); independent deviations dx_k of the inputs of a
sum move it by at most lam sqrt(sum_k W_jk^2 dx_k^2) with probability at least
1 - 2 exp(-lam^2 / 2) (Hoeffding).  lam = 8 makes either event less likely
than 1e-11 per element.
"""
import numpy as np

from oracle import surrogate as S

U = 2.0 ** -24
LAM = 8.0


def gamma(k, lam=None):
    if lam is None:
        return k * U / (1.0 - k * U)
    return float(np.expm1(lam * np.sqrt(k) * U + k * U * U / (1.0 - U)))


def spread(dx, Wabs, lam):
    """Deviation of x W^T from deviations dx of x (rows) through |W|."""
    if lam is None:
        return dx @ Wabs.T
    return lam * np.sqrt((dx * dx) @ (Wabs * Wabs).T)


def eps_silu(a):
    return (np.abs(a) + 8.0) * U


def eps_dsilu(a):
    return 2.0 * (np.abs(a) + 4.0) ** 2 * U


def ulp_bf16(x):
    """One bfloat16 unit at |x| (a normal value's 2^(e - 7))."""
    ax = np.maximum(np.abs(x), 2.0 ** -126)
    return 2.0 ** (np.floor(np.log2(ax)) - 7.0)


def flip_possible(v, delta):
    """Whether rounding v (taken to binary32) to bfloat16 can differ from
    rounding a value within delta of it: v lies within delta (plus one
    binary32 rounding) of a rounding midpoint."""
    v32 = np.asarray(v, dtype=np.float32)
    low = (v32.view(np.uint32) & 0xFFFF).astype(np.int64)
    ulp32 = np.spacing(np.abs(v32)).astype(np.float64)
    dist = np.abs(low - 0x8000) * ulp32
    return dist <= np.asarray(delta) + U * np.abs(v32.astype(np.float64))


def enter(h, dh, mode):
    """Value of an activation entering a product on the oracle's side, and
    the bound of the device's entering value's deviation from it (the two
    sides hold binary32 activations within dh + u|h| of each other).

    bf16: equal unless the rounding may flip (then one bfloat16 ulp).
    bf16x2: hi = bf16(v), lo = bf16(v - hi), v - hi exact.  While neither
    rounding can flip, lo moves with v and the entering values differ by the
    activations' difference; if lo may flip, by one more ulp of lo; if hi may
    flip, by at most the difference plus the two representation errors
    (each within 2^-18 |v|)."""
    d = dh + U * np.abs(h)
    if mode == "bf16":
        x = S._mfma_input(h, mode)
        return x, np.where(flip_possible(h, d), ulp_bf16(x), 0.0)
    v = np.asarray(h, dtype=np.float32)
    hi = S.bf16_rne(v)
    r = (v - hi).astype(np.float32)
    lo = S.bf16_rne(r)
    x = hi.astype(np.float64) + lo.astype(np.float64)
    hi_flip = flip_possible(v, d)
    lo_flip = flip_possible(r, d)
    dx = np.where(hi_flip, d + 2.0 ** -17 * (np.abs(h) + d),
                  np.where(lo_flip, d + 2.0 * ulp_bf16(np.maximum(np.abs(lo), np.abs(r))), d))
    return x, dx


def forward_bound(c, mode, lam=LAM):
    """Per-element deviation bounds (a_l, h_l, o) of the device forward from
    the oracle's forward in the same mode (cache c of S.forward).  Sums count
    their non-zero products: 5 inputs (x2: 10) in layer 1, 256 (x2: 512)
    after it."""
    W = c["W"]
    k2 = 2 if mode == "bf16x2" else 1
    x, _ = enter(c["u"], np.zeros_like(c["u"]), mode)   # u is binary32 on both sides
    da = {1: gamma(k2 * 5, lam) * (np.abs(x) @ np.abs(W["W1"]).T) + U * np.abs(c["a1"])}
    dh = {1: 1.1 * da[1] + eps_silu(c["a1"]) * np.abs(S.silu(c["a1"]))}
    for l in (2, 3):
        x, dx = enter(c[f"h{l - 1}"], dh[l - 1], mode)
        Wl = np.abs(W[f"W{l}"])
        da[l] = (spread(dx, Wl, lam) + gamma(k2 * 256, lam) * (np.abs(x) @ Wl.T)
                 + U * np.abs(c[f"a{l}"]))
        dh[l] = (dh[l - 1] + 2.0 ** -18 * np.abs(c[f"h{l - 1}"]) + 1.1 * da[l]
                 + eps_silu(c[f"a{l}"]) * np.abs(S.silu(c[f"a{l}"])) + U * np.abs(c[f"h{l}"]))
    x, dx = enter(c["h3"], dh[3], mode)
    W4 = np.abs(W["W4"])
    o = x @ W["W4"].T + W["b4"]
    do = spread(dx, W4, lam) + gamma(k2 * 256, lam) * (np.abs(x) @ W4.T) + U * np.abs(o)
    return da, dh, do


def grad_bound(parts, mode, n, lam=LAM):
    """Per-parameter bound of |device gradient - oracle's bf16-emulated
    gradient| (parts of S.loss_and_grad_bf16), flat in parameter order."""
    c, pre, rnd, dhv = parts["cache"], parts["pre"], parts["rnd"], parts["dh"]
    W = c["W"]
    da, dh_f, do = forward_bound(c, mode, lam)
    scale = float(np.float32(2.0) / np.float32(6.0 * n))
    # output error: (o - t) in binary32 from a deviating o, times the scale
    dpre = do * scale + 3.0 * U * np.abs(pre["dO"])
    e = {"dO": np.where(flip_possible(pre["dO"], dpre), ulp_bf16(rnd["dO"]), 0.0)}
    W4t = np.abs(W["W4"]).T
    d_dh = spread(e["dO"], W4t, lam) + gamma(6, lam) * (np.abs(rnd["dO"]) @ W4t.T)
    for l in (3, 2, 1):
        a = c[f"a{l}"]
        ds = S.dsilu(a)
        dpre = (np.abs(ds) * d_dh + np.abs(dhv[l]) * (0.5 * da[l] + eps_dsilu(a))
                + U * np.abs(pre[f"dA{l}"]))
        e[f"dA{l}"] = np.where(flip_possible(pre[f"dA{l}"], dpre), ulp_bf16(rnd[f"dA{l}"]), 0.0)
        if l > 1:
            Wl = np.abs(W[f"W{l}"])
            d_dh = (d_dh + spread(e[f"dA{l}"], Wl.T, lam)
                    + gamma(256, lam) * (np.abs(rnd[f"dA{l}"]) @ Wl) + U * np.abs(dhv[l - 1]))
    # activations entering the weight gradients as one bfloat16
    dev_h = {"u": np.zeros_like(c["u"]), "h1": dh_f[1], "h2": dh_f[2], "h3": dh_f[3]}
    for k, v in dev_h.items():
        e[k] = np.where(flip_possible(pre[k], v + U * np.abs(pre[k])), ulp_bf16(rnd[k]), 0.0)

    def gb(A, B):
        a, b = np.abs(rnd[A]), np.abs(rnd[B])
        G = rnd[A].T @ rnd[B]
        flips = spread(e[A].T, b.T, lam) + spread(a.T, e[B].T, lam) + e[A].T @ e[B]
        return flips + gamma(n, lam) * (a.T @ b) + 2.0 * U * np.abs(G)

    def bb(A):
        G = rnd[A].sum(0)
        ones = np.ones((1, e[A].shape[0]))
        fl = spread(e[A].T, ones, lam)[:, 0]
        return fl + gamma(n, lam) * np.abs(rnd[A]).sum(0) + 2.0 * U * np.abs(G)

    out = {"W4": gb("dO", "h3"), "b4": bb("dO"), "W3": gb("dA3", "h2"), "b3": bb("dA3"),
           "W2": gb("dA2", "h1"), "b2": bb("dA2"), "W1": gb("dA1", "u"), "b1": bb("dA1")}
    return np.concatenate([out[name].reshape(-1) for name, _ in S.SHAPES])
