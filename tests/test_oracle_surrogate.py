"""Pins of the surrogate oracle: bfloat16 rounding against torch's own
conversion, the network and its gradient against torch autograd and central
finite differences, Adam against closed forms and torch.optim.Adam, the
section's linear map against symplecticity and linearity, the Twiss
parameters against their defining invariants, and the gate against plain
tracking (no admitted particle is lost)."""
import math

import numpy as np
import pytest
import torch

from oracle import surrogate as S
from paper_1710_07350_amd import inputs

SIG = np.array(inputs.BEAM_SIGMAS)
HW = 6.0 * SIG
# central-difference step of the linear map, relative to the box half width:
# the best balance of truncation (sextupoles) and rounding (the bend's
# polar-frame update cancels terms of ~6 cm) on this section
H_REL = 1e-4


# ---------------------------------------------------------------- bfloat16
def test_bf16_rne_matches_torch_conversion():
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(200000) * np.exp(rng.uniform(-20, 20, 200000))).astype(np.float32)
    # exact ties: low 16 bits 0x8000 with even and odd kept parts
    bits = rng.integers(0x3F800000, 0x40800000, 2000, dtype=np.uint64).astype(np.uint32)
    ties = ((bits & 0xFFFF0000) | 0x8000).astype(np.uint32).view(np.float32)
    x = np.concatenate([x, ties, -ties, np.float32([0.0, -0.0, 1.0, 65504.0, 1e-30])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    got = S.bf16_rne(x)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_split_bf16x2_carries_sixteen_bits():
    rng = np.random.default_rng(4)
    x = rng.standard_normal(100000).astype(np.float32)
    hi, lo = S.split_bf16x2(x)
    assert np.array_equal(hi, S.bf16_rne(hi)) and np.array_equal(lo, S.bf16_rne(lo))
    err = np.abs(x.astype(np.float64) - hi.astype(np.float64) - lo.astype(np.float64))
    assert (err <= np.abs(x) * 2.0 ** -16).all()
    assert (np.abs(lo) <= np.abs(x) * 2.0 ** -8).all()


# ---------------------------------------------------------------- network
def torch_net(p64: np.ndarray):
    P = {k: torch.from_numpy(np.array(v, dtype=np.float64)).requires_grad_(True)
         for k, v in S.unpack(p64.copy()).items()}

    def f(u):
        u = u.clone()
        u[:, S.S_COORD] = 0.0
        h1 = torch.nn.functional.silu(torch.nn.functional.linear(u, P["W1"], P["b1"]))
        h2 = h1 + torch.nn.functional.silu(torch.nn.functional.linear(h1, P["W2"], P["b2"]))
        h3 = h2 + torch.nn.functional.silu(torch.nn.functional.linear(h2, P["W3"], P["b3"]))
        return torch.nn.functional.linear(h3, P["W4"], P["b4"])
    return f, P


def test_param_count():
    assert S.N_PARAM == 134918


def test_forward_matches_torch():
    p = S.init_params(1).astype(np.float64)
    P = S.unpack(p)
    rng = np.random.default_rng(5)
    for k in P:                       # non-zero biases exercise every term
        if k.startswith("b"):
            P[k][...] = rng.uniform(-0.3, 0.3, P[k].shape)
    u = rng.uniform(-1, 1, (64, 6))
    o = S.forward(p, u, "exact", round_weights=False)
    f, _ = torch_net(p)
    ref = f(torch.from_numpy(u)).detach().numpy()
    np.testing.assert_allclose(o, ref, rtol=1e-13, atol=1e-15)


def test_forward_rounds_weights_to_bf16():
    p = S.init_params(2)
    u = np.random.default_rng(6).uniform(-1, 1, (16, 6))
    q = S.bf16_rne(p).astype(np.float64)       # every entry rounded, biases too
    P = S.unpack(q)
    for k in ("b1", "b2", "b3", "b4"):
        P[k][...] = S.unpack(p)[k]
    a = S.forward(p, u, "exact", round_weights=True)
    b = S.forward(q, u, "exact", round_weights=False)
    assert np.array_equal(a, b)


def test_gradient_matches_torch_autograd():
    p = S.init_params(3).astype(np.float64)
    rng = np.random.default_rng(7)
    u = rng.uniform(-1, 1, (32, 6))
    t = rng.standard_normal((32, 6)) * 0.1
    loss, g = S.loss_and_grad(p, u, t, round_weights=False)
    f, P = torch_net(p)
    L = ((f(torch.from_numpy(u)) - torch.from_numpy(t)) ** 2).sum() / (6 * 32)
    L.backward()
    ref = np.concatenate([P[k].grad.numpy().reshape(-1) for k, _ in S.SHAPES])
    assert loss == pytest.approx(float(L.detach()), rel=1e-13)
    np.testing.assert_allclose(g, ref, rtol=1e-11, atol=1e-16)


def test_gradient_matches_central_differences():
    p = S.init_params(4).astype(np.float64)
    P = S.unpack(p)
    rng = np.random.default_rng(8)
    for k in P:
        if k.startswith("b"):
            P[k][...] = rng.uniform(-0.2, 0.2, P[k].shape)
    u = rng.uniform(-1, 1, (16, 6))
    t = rng.standard_normal((16, 6)) * 0.1
    _, g = S.loss_and_grad(p, u, t, round_weights=False)
    idx = np.concatenate([rng.choice(S.N_PARAM, 300, replace=False),
                          [0, 1540, 1791, S.N_PARAM - 1, S.N_PARAM - 7]])
    h = 1e-6
    for i in idx:
        q = p.copy()
        q[i] += h
        lp, _ = S.loss_and_grad(q, u, t, round_weights=False)
        q[i] -= 2 * h
        lm, _ = S.loss_and_grad(q, u, t, round_weights=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(abs(g[i]), 1e-4), (i, fd, g[i])


def test_structural_zeros():
    """s never enters (its W1 column has zero gradient) and the delta output
    receives no gradient when its target and weights are zero."""
    p = S.init_params(5).astype(np.float64)
    rng = np.random.default_rng(9)
    u = rng.uniform(-1, 1, (32, 6))
    t = rng.standard_normal((32, 6)) * 0.1
    t[:, S.D_COORD] = 0.0
    _, g = S.loss_and_grad(p, u, t, round_weights=False)
    G = S.unpack(g)
    assert (G["W1"][:, S.S_COORD] == 0.0).all()
    u2 = u.copy()
    u2[:, S.S_COORD] = rng.uniform(-1, 1, 32)
    assert np.array_equal(S.forward(p, u, "bf16x2"), S.forward(p, u2, "bf16x2"))


def test_bf16_modes_are_close_to_exact():
    p = S.init_params(6)
    u = np.random.default_rng(10).uniform(-1, 1, (256, 6))
    e = S.forward(p, u, "exact")
    x2 = S.forward(p, u, "bf16x2")
    x1 = S.forward(p, u, "bf16")
    scale = np.abs(e).max()
    assert np.abs(x2 - e).max() <= 1e-4 * scale
    assert 1e-4 * scale < np.abs(x1 - e).max() <= 3e-2 * scale


# ---------------------------------------------------------------- Adam
def _bf16_t(x):
    return torch.from_numpy(S.bf16_rne(x.detach().numpy().astype(np.float32)).astype(np.float64))


class _RoundGrad(torch.autograd.Function):
    """Identity forward; the incoming gradient rounded to bfloat16."""

    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return _bf16_t(g)


class _Lin(torch.autograd.Function):
    """x W^T + b with the input entering as bfloat16 x2 (forward) and as one
    bfloat16 in the weight gradient."""

    @staticmethod
    def forward(ctx, h, W, b):
        x = torch.from_numpy(S._mfma_input(h.detach().numpy(), "bf16x2"))
        ctx.save_for_backward(_bf16_t(h), W)
        return x @ W.T + b

    @staticmethod
    def backward(ctx, g):
        hb, W = ctx.saved_tensors
        return g @ W, g.T @ hb, g.sum(0)


def test_bf16_emulated_gradient_matches_autograd_with_rounding_hooks():
    """The rounding points of loss_and_grad_bf16 re-expressed as autograd
    functions (round the gradient at each pre-activation and at the output,
    bfloat16 inputs in the weight gradients): torch derives the chain and the
    skip sums itself; the two agree to summation order."""
    p = S.init_params(5)
    P = S.unpack(p)
    rng = np.random.default_rng(15)
    for k in ("b1", "b2", "b3"):
        P[k][...] = rng.uniform(-0.3, 0.3, P[k].shape).astype(np.float32)
    n = 256
    u = rng.uniform(-1, 1, (n, 6)).astype(np.float32).astype(np.float64)
    u[:, S.S_COORD] = 0.0
    t = rng.standard_normal((n, 6)) * 0.2
    t[:, S.D_COORD] = 0.0
    loss, g, parts = S.loss_and_grad_bf16(p, u, t)
    W = {k: torch.from_numpy(v.copy()).requires_grad_(True) for k, v in S.weights(p).items()}
    ut = torch.from_numpy(u)
    a1 = _RoundGrad.apply(_Lin.apply(ut, W["W1"], W["b1"]))
    h1 = torch.nn.functional.silu(a1)
    a2 = _RoundGrad.apply(_Lin.apply(h1, W["W2"], W["b2"]))
    h2 = h1 + torch.nn.functional.silu(a2)
    a3 = _RoundGrad.apply(_Lin.apply(h2, W["W3"], W["b3"]))
    h3 = h2 + torch.nn.functional.silu(a3)
    o = _RoundGrad.apply(_Lin.apply(h3, W["W4"], W["b4"]))
    c = float(np.float32(2.0) / np.float32(6.0 * n)) / 2.0
    (((o - torch.from_numpy(t)) ** 2).sum() * c).backward()
    assert loss == pytest.approx(float(((o.detach().numpy() - t) ** 2).sum() / (6.0 * n)), rel=1e-14)
    G = S.unpack(g)
    for name, _ in S.SHAPES:
        ref = W[name].grad.numpy()
        diff = np.abs(G[name] - ref)
        scale = np.abs(ref).max()
        assert (diff <= 1e-12 * scale).mean() > 0.999, name
        assert diff.max() <= 2.0 ** -7 * scale, name
    # the rounding is felt: the emulated gradient is not the exact one
    _, gx = S.loss_and_grad(p, u, t)
    rel = np.linalg.norm(g - gx) / np.linalg.norm(gx)
    assert 1e-5 < rel < 1e-2


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(11)
    w = rng.standard_normal(1000).astype(np.float32)
    g = rng.standard_normal(1000).astype(np.float32)
    z = np.zeros(1000, np.float32)
    lr = 1e-3
    w1, m1, v1 = S.adam(w, z, z, g, 1, lr)
    g64 = g.astype(np.float64)
    ref = w.astype(np.float64) - lr * g64 / (np.abs(g64) + 1e-8)
    np.testing.assert_allclose(w1, ref, rtol=2e-7, atol=1e-9)
    np.testing.assert_allclose(m1, 0.1 * g64, rtol=1e-6)


def test_adam_constant_gradient_moves_linearly():
    w = np.float32([0.5, -2.0, 3.0])
    g = np.float32([0.25, -1.0, 4.0])
    m = np.zeros(3, np.float32)
    v = np.zeros(3, np.float32)
    lr = 1e-4
    for t in range(1, 201):
        w, m, v = S.adam(w, m, v, g, t, lr)
    ref = np.float64([0.5, -2.0, 3.0]) - 200 * lr * np.sign(g)
    # w is stored in binary32: each of the 200 steps rounds it by <= half an ulp
    tol = 200 * 0.5 * np.spacing(np.abs(w)).astype(np.float64) + 1e-9
    assert (np.abs(w - ref) <= tol).all()


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(12)
    w = rng.standard_normal(500).astype(np.float32)
    m = np.zeros(500, np.float32)
    v = np.zeros(500, np.float32)
    tw = torch.from_numpy(w.astype(np.float64)).requires_grad_(True)
    opt = torch.optim.Adam([tw], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.standard_normal(500).astype(np.float32)
        w, m, v = S.adam(w, m, v, g, t, 3e-3)
        tw.grad = torch.from_numpy(g.astype(np.float64))
        opt.step()
    np.testing.assert_allclose(w, tw.detach().numpy(), rtol=1e-6, atol=1e-7)


# ---------------------------------------------------------------- linear map
def section():
    return inputs.ring_lattice(seed=0)[:100]


def to_canon(z):
    x, xp, y, yp, s, d = z
    f = (1.0 + d) / math.sqrt(1.0 + xp * xp + yp * yp)
    return np.array([x, xp * f, y, yp * f, -s, d])


def test_section_linear_map_is_symplectic(orc):
    C, R = S.linear_map(orc, section(), HW, H_REL)
    # canonical Jacobian: d canon / d slopes at the output point C, times R,
    # times the inverse of the same at the input origin
    Jout = np.zeros((6, 6))
    for k in range(6):
        e = np.zeros(6)
        e[k] = 1e-7
        Jout[:, k] = (to_canon(C + e) - to_canon(C - e)) / 2e-7
    Jin = np.diag([1.0, 1.0, 1.0, 1.0, -1.0, 1.0])
    M = Jout @ R @ np.linalg.inv(Jin)
    J = np.zeros((6, 6))
    for i in range(3):
        J[2 * i, 2 * i + 1], J[2 * i + 1, 2 * i] = 1.0, -1.0
    assert np.abs(M.T @ J @ M - J).max() < 1e-7
    # delta passes unchanged; s does not act on anything
    assert np.array_equal(R[5], [0, 0, 0, 0, 0, 1.0]) and C[5] == 0.0
    assert np.array_equal(R[[0, 1, 2, 3, 5], 4], np.zeros(5)) and abs(R[4, 4] - 1.0) < 1e-9


def test_section_linear_map_is_the_first_order_part(orc):
    C, R = S.linear_map(orc, section(), HW, H_REL)
    rng = np.random.default_rng(13)
    v = rng.uniform(-1, 1, 6) * HW
    errs = []
    for eps in (1e-3, 5e-4):
        z = np.stack([eps * v, np.zeros(6)], axis=1)
        b = orc.Beam(z, np.arange(2, dtype=np.uint32), np.full(2, -1, np.int64))
        orc.track(b, section(), 1)
        errs.append(np.abs(b.z[:, 0] - C - R @ (eps * v)).max())
    # the remainder is second order: halving eps quarters it
    assert 3.5 < errs[0] / errs[1] < 4.5


# ---------------------------------------------------------------- gate
_PARTIAL = []


def partial_maps(orc):
    """Linear maps from the section entrance to every element exit."""
    if not _PARTIAL:
        sec = section()
        _PARTIAL.extend(S.linear_map(orc, sec[:k + 1], HW, H_REL)[1] for k in range(len(sec)))
    return _PARTIAL


def test_twiss_invariants(orc):
    C, R = S.linear_map(orc, section(), HW, H_REL)
    for i in (0, 2):
        a, b, g, eta, etap = S.twiss(R, i)
        # beta gamma - alpha^2 = det of the block = 1 up to the difference error
        assert b > 0 and abs(b * g - a * a - 1.0) < 1e-7
        T = np.array([[b, -a], [-a, g]])
        M = R[i:i + 2, i:i + 2]
        np.testing.assert_allclose(M @ T @ M.T, T, rtol=1e-7, atol=1e-9)
        if i == 0:
            np.testing.assert_allclose(M @ [eta, etap] + R[i:i + 2, 5], [eta, etap],
                                       rtol=1e-9, atol=1e-12)
    # the last partial map is the section map itself
    assert np.array_equal(partial_maps(orc)[-1], R)


def test_gate_admits_only_survivors(orc):
    C, R = S.linear_map(orc, section(), HW, H_REL)
    g = S.gate_constants(R, partial_maps(orc), HW, 0.5, 10e-3, 5e-3)
    n = 100000
    z = inputs.uniform_box_beam(n, seed=21, half_widths=HW)["z"]
    adm = S.gate(z, g)
    assert 0.001 < adm.mean() < 0.05
    b = orc.Beam(z[:, adm], np.arange(int(adm.sum()), dtype=np.uint32),
                 np.full(int(adm.sum()), -1, np.int64))
    orc.track(b, section(), 1)
    assert (b.lost_at < 0).all()
    # a larger margin admits a subset
    g2 = S.gate_constants(R, partial_maps(orc), HW, 0.6, 10e-3, 5e-3)
    adm2 = S.gate(z, g2)
    assert (adm2 <= adm).all() and adm2.sum() < adm.sum()
    # the box: outside +-hw is never admitted, whatever the amplitude
    z2 = np.zeros((6, 3))
    z2[5] = [1.01 * HW[5], -1.01 * HW[5], 0.1 * HW[5]]
    assert list(S.gate(z2, g)) == [False, False, True]


# ---------------------------------------------------------------- sampler box
def _gate_and_widths(orc, margin=0.5):
    C, R = S.linear_map(orc, section(), HW, H_REL)
    g = S.gate_constants(R, partial_maps(orc), HW, margin, 10e-3, 5e-3)
    return g, S.sample_widths(g, 10e-3, 5e-3)


def _to_box_edge(v, hw):
    """Scale each ray (column) so that its largest |v_k| / hw_k is 1: at
    t = 1 it touches the training box, beyond it the gate refuses."""
    return v / (np.abs(v) / np.asarray(hw)[:, None]).max(axis=0)


def _boundary(g, v, iters=70):
    """Outermost admitted point along each ray t v, 0 < t <= 1, for rays
    scaled to the box edge: the admitted set is star-shaped about the origin
    (the box is, and the amplitudes sqrt(J) and |delta| scale linearly with
    t), so bisection finds its edge."""
    v = _to_box_edge(v, g["hw"])
    lo = np.zeros(v.shape[1])
    hi = np.full(v.shape[1], 1.0 + 1e-9)
    assert not S.gate(v * hi, g).any()
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        ok = S.gate(v * mid, g)
        lo = np.where(ok, mid, lo)
        hi = np.where(ok, hi, mid)
    return v * lo


def _extremal_rays(g):
    """Rays through the points of the Courant--Snyder ellipses where one
    coordinate is extreme: on gamma u^2 + 2 alpha u u' + beta u'^2 = J the
    largest u is sqrt(J beta) at u' = -alpha sqrt(J/beta), the largest u' is
    sqrt(J gamma) at u = -alpha sqrt(J/gamma); the pure dispersion ray
    (eta, eta', 0, 0, 0, 1) has no betatron amplitude at all.  Mixtures of
    the x-extreme betatron ray and the dispersion ray (each scaled to one
    unit of the gate's x amplitude) cover the shared budget."""
    bx, gx, ax = g["bx"], g["gx"], g["ax2"] / 2.0
    by, gy, ay = g["by"], g["gy"], g["ay2"] / 2.0
    bet_x = np.array([math.sqrt(bx), -ax / math.sqrt(bx), 0, 0, 0, 0]) / math.sqrt(g["bhx"])
    bet_xp = np.array([-ax / math.sqrt(gx), math.sqrt(gx), 0, 0, 0, 0]) / math.sqrt(g["bhx"])
    disp = np.array([g["eta"], g["etap"], 0, 0, 0, 1.0]) / g["eh"]
    rays = [np.array([0, 0, math.sqrt(by), -ay / math.sqrt(by), 0, 0]),
            np.array([0, 0, -ay / math.sqrt(gy), math.sqrt(gy), 0, 0]), disp]
    sx = 1.0 if g["eta"] >= 0 else -1.0
    sxp = 1.0 if g["etap"] >= 0 else -1.0
    for c in np.linspace(0.0, 1.0, 41):
        rays.append((1 - c) * bet_x + c * sx * disp)
        rays.append((1 - c) * bet_xp + c * sxp * disp)
    rays += [-r for r in rays]
    return np.array(rays, dtype=float).T


def test_sampler_box_contains_every_admitted_point(orc):
    """sample_widths bounds every coordinate of every admitted point: points
    on the edge of the admitted set (bisection along random rays and along the
    rays of the extremal ellipse points), and admitted points of a uniform box
    wider than the sampler's, all lie within the half widths."""
    g, sw = _gate_and_widths(orc)
    rng = np.random.default_rng(31)
    n = 40000
    v = rng.standard_normal((6, n))
    v[4] = 0.0
    v *= HW[:, None]
    # rays weighted towards a few coordinates at a time as well
    v2 = rng.standard_normal((6, n)) * (rng.random((6, n)) < 0.4) * HW[:, None]
    v2[4] = 0.0
    v2 = v2[:, np.abs(v2).sum(0) > 0]
    edge = _boundary(g, np.concatenate([v, v2, _extremal_rays(g)], axis=1))
    assert S.gate(edge, g).all()
    for k in (0, 1, 2, 3, 5):
        assert (np.abs(edge[k]) <= sw[k]).all(), (k, np.abs(edge[k]).max(), sw[k])
    wide = np.minimum(1.5 * sw, HW)
    wide[4] = HW[4]
    box = inputs.uniform_box_beam(400000, seed=32, half_widths=wide)["z"]
    adm = S.gate(box, g)
    assert adm.sum() > 2000
    for k in (0, 1, 2, 3, 5):
        assert (np.abs(box[k, adm]) <= sw[k]).all()


def test_sampler_box_is_not_loose(orc):
    """The half widths are reached.  With the training box widened tenfold
    (so that only the amplitude bound limits), the edge points of the
    extremal rays reach the uncapped widths of y, y' and delta (the bound is
    exact there, up to the 1e-6 padding), and those of x and x' at least
    half-way (their bound adds the betatron and the dispersion extremes,
    which the gate makes share one amplitude budget)."""
    g, sw = _gate_and_widths(orc)
    gw = dict(g, hw=tuple(10.0 * HW))
    sww = S.sample_widths(gw, 10e-3, 5e-3)
    assert (sww[[0, 1, 2, 3, 5]] < 10.0 * HW[[0, 1, 2, 3, 5]]).all()
    np.testing.assert_array_equal(np.minimum(sww, HW), sw)
    edge = _boundary(gw, _extremal_rays(gw))
    reach = np.abs(edge).max(axis=1) / sww
    assert (reach[[0, 1, 2, 3, 5]] <= 1.0).all()
    for k in (2, 3, 5):
        assert reach[k] > 1 - 1e-5, (k, reach[k])
    for k in (0, 1):
        assert reach[k] > 0.5, (k, reach[k])
    # a larger margin shrinks every width
    g2 = S.gate_constants(S.linear_map(orc, section(), HW, H_REL)[1], partial_maps(orc),
                          10.0 * HW, 0.7, 10e-3, 5e-3)
    sw2 = S.sample_widths(g2, 10e-3, 5e-3)
    assert (sw2[[0, 1, 2, 3, 5]] < sww[[0, 1, 2, 3, 5]]).all()


def _synthetic_gate(rng, g0):
    """Gate constants of an arbitrary lattice position: random Twiss
    parameters (beta gamma - alpha^2 = 1), dispersion, and maxima over the
    section at or above the entrance values, as gate_constants produces."""
    g = dict(g0, hw=tuple(10.0 * HW))
    for pl in ("x", "y"):
        b = rng.uniform(1.0, 20.0)
        a = rng.uniform(-2.0, 2.0)
        g["b" + pl] = b
        g["a" + pl + "2"] = 2.0 * a
        g["g" + pl] = (1.0 + a * a) / b
        g["bh" + pl] = b * rng.uniform(1.0, 4.0)
    g["eta"] = rng.uniform(-3.0, 3.0)
    g["etap"] = rng.uniform(-0.5, 0.5)
    g["eh"] = abs(g["eta"]) * rng.uniform(1.0, 3.0) + 0.1
    return g


def test_sampler_box_contains_admitted_points_of_any_lattice(orc):
    """Containment and reach for random gate constants (the section's own
    constants leave the dispersion term of x inside the cap of the box)."""
    g0, _ = _gate_and_widths(orc)
    rng = np.random.default_rng(33)
    for _ in range(12):
        g = _synthetic_gate(rng, g0)
        sw = S.sample_widths(g, 10e-3, 5e-3)
        v = rng.standard_normal((6, 4000)) * HW[:, None]
        v[4] = 0.0
        edge = _boundary(g, np.concatenate([v, _extremal_rays(g)], axis=1))
        reach = np.abs(edge).max(axis=1) / sw
        assert (reach[[0, 1, 2, 3, 5]] <= 1.0).all(), reach
        assert (reach[[2, 3, 5]] > 1 - 1e-5).all(), reach
        assert (reach[[0, 1]] > 0.5).all(), reach


class _Words:
    """Stand-in generator returning fixed words, to pin the word -> uniform
    -> coordinate map of the sampler."""

    def __init__(self, w):
        self.w = w

    def philox4x32_10(self, ctr, key):
        return list(self.w[:4]) if ctr[3] == 0 else list(self.w[4:])


def test_sampler_draw_maps_words_to_the_open_box():
    sw = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0])
    lo = S.draw(_Words([0] * 8), sw, 0, 0)
    hi = S.draw(_Words([0xFFFFFFFF] * 8), sw, 0, 0)
    mid = S.draw(_Words([0x7FFFFFFF] * 8), sw, 0, 0)
    q = 2.0 ** -32
    np.testing.assert_array_equal(lo, -(1.0 - q) * sw)
    np.testing.assert_array_equal(hi, (1.0 - q) * sw)
    np.testing.assert_array_equal(mid, -q * sw * 0.0 + (2.0 * (0x7FFFFFFF + 0.5) * q - 1.0) * sw)
    # word k of the two blocks feeds coordinate k
    w = list(range(1000, 1008))
    z = S.draw(_Words(w), sw, 0, 0)
    np.testing.assert_array_equal(z, [(2.0 * ((w[k] + 0.5) * q) - 1.0) * sw[k] for k in range(6)])


def test_sampler_draws_are_uniform_and_independent(orc):
    from scipy import stats
    g, sw = _gate_and_widths(orc)
    n = 6000
    Z = np.array([S.draw(orc, sw, 5, c) for c in range(n)]).T
    assert (np.abs(Z) < sw[:, None]).all()
    U = (Z / sw[:, None] + 1.0) / 2.0
    for k in range(6):
        assert stats.kstest(U[k], "uniform").pvalue > 1e-3, k
    C = np.corrcoef(U)
    assert np.abs(C - np.eye(6)).max() < 0.06
    # other seeds and candidates beyond 2^32 give other points
    assert not np.array_equal(S.draw(orc, sw, 5, 7), S.draw(orc, sw, 6, 7))
    assert not np.array_equal(S.draw(orc, sw, 5, 7), S.draw(orc, sw, 5, 7 + 2 ** 32))


# ---------------------------------------------------------------- error bounds
def _f32_network(p, u, t, mode):
    """A binary32 evaluation with the device's structure: bfloat16 operands
    (activations split hi + lo in bf16x2 mode), binary32 products and sums,
    binary32 SiLU from exp2 and a reciprocal, the skip path read back as
    hi + lo; then the backward with the same rounding points as the oracle's
    emulation.  Returns (o, flat gradient)."""
    f32 = np.float32
    W = {k: v.astype(f32) for k, v in S.weights(p).items()}

    def split(h):
        hi = S.bf16_rne(h)
        lo = S.bf16_rne((h - hi).astype(f32))
        return hi, lo

    def mm(h, Wm):
        hi, lo = split(h)
        if mode == "bf16x2":
            return (hi @ Wm.T + lo @ Wm.T).astype(f32)
        return (hi @ Wm.T).astype(f32)

    def sig(a):
        return (f32(1.0) / (f32(1.0) + np.exp2(a * f32(-1.4426950408889634)))).astype(f32)

    u32 = u.astype(f32)
    a1 = (mm(u32, W["W1"]) + W["b1"]).astype(f32)
    h1 = (a1 * sig(a1)).astype(f32)
    a2 = (mm(h1, W["W2"]) + W["b2"]).astype(f32)
    hi, lo = split(h1)
    h2 = ((hi + lo) + a2 * sig(a2)).astype(f32)
    a3 = (mm(h2, W["W3"]) + W["b3"]).astype(f32)
    hi, lo = split(h2)
    h3 = ((hi + lo) + a3 * sig(a3)).astype(f32)
    o = (mm(h3, W["W4"]) + W["b4"]).astype(f32)
    n = u.shape[0]
    scale = f32(2.0) / f32(6.0 * n)
    dO = S.bf16_rne(((o - t.astype(f32)) * scale).astype(f32))
    dh = (dO @ W["W4"]).astype(f32)
    g = {"W4": dO.T @ S.bf16_rne(h3), "b4": dO.sum(0)}
    for l, a, hin in ((3, a3, h2), (2, a2, h1), (1, a1, u32)):
        s = sig(a)
        dA = S.bf16_rne((dh * (s * (f32(1.0) + a * (f32(1.0) - s)))).astype(f32))
        g[f"W{l}"] = (dA.T @ S.bf16_rne(hin)).astype(f32)
        g[f"b{l}"] = dA.sum(0, dtype=f32)
        if l > 1:
            dh = (dh + dA @ W[f"W{l}"]).astype(f32)
    flat = np.concatenate([np.asarray(g[name], dtype=np.float64).reshape(-1) for name, _ in S.SHAPES])
    return o.astype(np.float64), flat


@pytest.mark.parametrize("lam", [None, 8.0])
@pytest.mark.parametrize("mode", ["bf16x2", "bf16"])
def test_mlp_bounds_cover_a_binary32_evaluation(mode, lam):
    """The element-wise bounds the GPU tests use (tests/mlp_bounds.py) hold
    for an independent binary32 evaluation on the CPU: every output and every
    gradient element within its bound, and the bounds are not vacuous."""
    import mlp_bounds as MB
    p = S.init_params(8)
    P = S.unpack(p)
    rng = np.random.default_rng(18)
    for k in ("b1", "b2", "b3"):
        P[k][...] = rng.uniform(-0.3, 0.3, P[k].shape).astype(np.float32)
    n = 512
    u = rng.uniform(-1, 1, (n, 6)).astype(np.float32).astype(np.float64)
    u[:, S.S_COORD] = 0.0
    t = (rng.standard_normal((n, 6)) * 0.3).astype(np.float32).astype(np.float64)
    t[:, S.D_COORD] = 0.0
    o_ref, c = S.forward(p, u, mode, cache=True)
    _, _, do = MB.forward_bound(c, mode, lam)
    o32, g32 = _f32_network(p, u, t, mode)
    err = np.abs(o32[:, :5] - o_ref[:, :5])
    assert (err <= do[:, :5]).all(), (err / do[:, :5]).max()
    _, g_emu, parts = S.loss_and_grad_bf16(p, u, t, mode)
    bound = MB.grad_bound(parts, mode, n, lam)
    gerr = np.abs(g32 - g_emu)
    bad = gerr > bound
    assert not bad.any(), (bad.sum(), np.nonzero(bad)[0][:10])
    print(f"{mode} lam={lam}: output bound median {np.median(do[:, :5]):.2e} "
          f"(error max {err.max():.2e}, max err/bound {(err / do[:, :5]).max():.3f}); "
          f"gradient max err/bound {(gerr / np.maximum(bound, 1e-300)).max():.3f}")
