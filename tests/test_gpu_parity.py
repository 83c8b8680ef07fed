"""Parity of the HIP path with the CPU oracle on identical seeded inputs.

Binary64 tracking, loss records, survivor order, histogram counts and
Philox streams are bit-exact; moments agree to 1e-12 of the beam scale; the
FP32 matrix-core wake convolution stays inside its rounding-error bound.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1710_07350_amd import binding as B
from paper_1710_07350_amd import inputs
from paper_1710_07350_amd.inputs import Element

from helpers import assert_bit_exact, moments_close, rel_err, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

WIDE = (2e-3, 2e-4, 2e-3, 2e-4, 1e-3, 1e-3)   # wide enough to lose particles


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


# ------------------------------------------------------------------ FODO
def test_fodo_parity_with_moments(torch):
    lat = inputs.fodo_lattice()
    d = inputs.gaussian_beam(10_000, seed=0, sigmas=WIDE)
    g = run_gpu(lat, d, 100, moments=True)
    r = run_oracle(lat, d, 100, moments=True)
    assert 0 < r["n_alive"] < 10_000
    assert_bit_exact(g, r)
    moments_close(g["moments"], r["moments"])


def test_fodo_config_beam(torch):
    """The FODO channel's own configuration: 1e4 particles with the sigmas
    (1 mm, 0.1 mrad, 1 mm, 0.1 mrad, 1 mm, 1e-3), seed 0, 100 passes, moments
    after every pass; bit-exact with the oracle."""
    lat = inputs.fodo_lattice()
    d = inputs.gaussian_beam(10_000, seed=0)
    assert np.allclose(d["z"].std(axis=1), inputs.BEAM_SIGMAS, rtol=0.03)
    g = run_gpu(lat, d, 100, moments=True)
    r = run_oracle(lat, d, 100, moments=True)
    assert 0 < r["n_alive"] <= 10_000
    assert_bit_exact(g, r)
    moments_close(g["moments"], r["moments"])


@pytest.mark.parametrize("kw", [dict(passes_per_launch=1), dict(passes_per_launch=7),
                                dict(max_elems_per_launch=5), dict(max_elems_per_launch=1),
                                dict(max_elems_per_launch=1, run_nt=1),
                                dict(max_elems_per_launch=2, run_nt=1, run_ppt=4, run_blocks=3),
                                dict(max_elems_per_launch=3, run_nt=-1, run_ppt=8)])
def test_fodo_fusion_depth_does_not_change_results(torch, kw):
    """Fusion depth, streaming stores and launch shape change traffic, never
    results; with losses in early runs, later runs skip the lost slots."""
    lat = inputs.fodo_lattice()
    d = inputs.gaussian_beam(3000, seed=4, sigmas=WIDE)
    r = run_oracle(lat, d, 12)
    g = run_gpu(lat, d, 12, **kw)
    assert_bit_exact(g, r)


@pytest.mark.parametrize("n", [1, 63, 255, 257, 1000, 4099])
def test_ragged_sizes(torch, n):
    lat = inputs.fodo_lattice(ncells=3)
    d = inputs.gaussian_beam(n, seed=n, sigmas=WIDE)
    assert_bit_exact(run_gpu(lat, d, 9, moments=True), run_oracle(lat, d, 9, moments=True))


def test_every_particle_lost(torch):
    lat = inputs.fodo_lattice(ncells=2, aper=1e-4)
    d = inputs.gaussian_beam(2000, seed=2, sigmas=WIDE)
    g = run_gpu(lat, d, 4, moments=True)
    r = run_oracle(lat, d, 4, moments=True)
    assert r["n_alive"] == 0
    assert_bit_exact(g, r)
    assert (g["moments"][-1] == 0).all() and (r["moments"][-1] == 0).all()


def test_zero_slot_beam_is_a_no_op(torch):
    """n_total = 0 with valid device pointers: tracking (moments requested)
    and the three reorderings enqueue nothing; the moments call reports
    n = 0 and zero means and second moments."""
    d = inputs.gaussian_beam(1, seed=1)
    beam = B.Beam.from_inputs(d)
    before = beam.host()
    ws = B.Workspace(1)
    lat = B.Lattice(inputs.fodo_lattice(ncells=2, aper=1e-4))
    mom = torch.full((3, 28), 7.0, dtype=torch.float64, device="cuda")
    beam.n = 0
    B.track(beam, lat, 3, ws, moments=mom)
    for mode in (B.COMPACT_STABLE, B.COMPACT_SWAP, B.COMPACT_SORT):
        B.compact_lost(beam, ws, mode=mode)
    m = B.moments(beam, ws).cpu().numpy()
    beam.n = 1
    after = beam.host()
    for k in ("z", "id", "lost_at", "n_alive"):
        assert np.array_equal(before[k], after[k])
    assert (mom.cpu().numpy() == 7.0).all()
    assert (m == 0).all()


def test_first_pass_offset_and_markers(torch):
    lat = inputs.fodo_lattice(ncells=2) + [Element("MARKER", aperture="ELLIPSE", ax=4e-3, ay=3e-3)]
    d = inputs.gaussian_beam(4000, seed=9, sigmas=WIDE)
    g = run_gpu(lat, d, 3, first_pass=40)
    r = run_oracle(lat, d, 3, first_pass=40)
    assert_bit_exact(g, r)
    lost = g["lost_at"][g["lost_at"] >= 0]
    assert lost.size and ((lost >> 32) >= 40).all()


# ------------------------------------------------------------------ ring
@pytest.mark.parametrize("ppt", [0, 2])
def test_ring_subset_parity(torch, ppt):
    lat = inputs.ring_lattice(seed=0)
    d = inputs.gaussian_beam(2000, seed=3, sigmas=(3e-3, 3e-4, 2e-3, 2e-4, 1e-3, 1e-3))
    g = run_gpu(lat, d, 30, seed=77, moments=True, run_ppt=ppt)
    r = run_oracle(lat, d, 30, seed=77, moments=True)
    assert 0 < r["n_alive"] < 2000
    assert_bit_exact(g, r)
    moments_close(g["moments"], r["moments"])


def test_ring_one_thousand_turns_in_one_call(torch):
    """The storage ring's configured run length in one trk_track call: 1000
    turns with moments after every turn at the default fusion (16 turns per
    launch, lazy compaction across the whole call, so late launches skip
    hundreds of turns' worth of lost slots), on a 4000-particle id subset of
    the configured 1e6-particle beam (seed 0; kicks keyed by id, so the
    subset's particles follow the same trajectories as in the full beam).
    Bit-exact coordinates, loss records and order; moments within 1e-12."""
    lat = inputs.ring_lattice(seed=0)
    full = inputs.gaussian_beam(1_000_000, seed=0)
    pick = np.sort(np.random.default_rng(11).choice(1_000_000, 4000, replace=False))
    d = {"z": np.ascontiguousarray(full["z"][:, pick]), "id": full["id"][pick],
         "lost_at": full["lost_at"][pick]}
    g = run_gpu(lat, d, 1000, seed=7, moments=True)
    r = run_oracle(lat, d, 1000, seed=7, moments=True)
    assert 0 < r["n_alive"] < 4000
    lost_turns = r["lost_at"][r["lost_at"] >= 0] >> 32
    assert lost_turns.max() >= 16              # losses in more than one launch
    assert_bit_exact(g, r)
    moments_close(g["moments"], r["moments"])


def test_ring_multistep_elements(torch):
    lat = inputs.ring_lattice(seed=5, ncells=4, nsteps=3)
    d = inputs.gaussian_beam(1500, seed=6)
    assert_bit_exact(run_gpu(lat, d, 5, seed=1), run_oracle(lat, d, 5, seed=1))


def test_generic_map_and_octupole(torch):
    rng = np.random.default_rng(12)
    c = np.zeros(168)
    c[:6] = rng.normal(0, 1e-5, 6)
    c[6:42] = (np.eye(6) + rng.normal(0, 0.05, (6, 6))).ravel()
    c[42:] = rng.normal(0, 0.3, 126) * (rng.random(126) < 0.5)
    lat = [Element("MAP2", coef=c, aperture="RECT", ax=4e-3, ay=4e-3),
           Element("MULT", k=300.0, order=3), Element("QUAD", L=0.3, k=0.0),
           Element("EDRIFT", L=0.7, aperture="RECT", ax=4e-3, ay=4e-3)]
    d = inputs.gaussian_beam(3000, seed=8, sigmas=WIDE)
    assert_bit_exact(run_gpu(lat, d, 6), run_oracle(lat, d, 6))


# ------------------------------------------------------------------ bunch compressor
def bc_bound_on_delta(d, lat, n0):
    """|delta_fp32 - delta_fp64| bound after the 8 wake steps: each V value
    errs by at most (nbins + 2) 2^-24 sum_j c_j |W[i-j]| (FP32 products, sums
    and table rounding), interpolation is a convex combination, and the RF
    kicks only scale earlier errors by P/P' < 1."""
    nb = lat[1].nbins
    rg, cnt = oracle.histogram(d["z"][4], d["lost_at"], nb)
    w = oracle.wake_table(rg[0], rg[1], nb, lat[1].wake_tau0, lat[1].wake_omega)
    scale = np.convolve(cnt.astype(float), np.abs(w))[:nb]
    bound_v = (nb + 2) * 2.0 ** -24 * scale.max()
    P = inputs.BC_P0_EV
    tot = 0.0
    for e in lat:
        if e.kind == "RFCA":
            P = P + e.volt * math.cos(e.phase)
        if e.kind == "WAKE":
            tot += oracle.wake_kfac(e.charge, n0, e.wake_A, P) * bound_v
    return tot


@pytest.mark.parametrize("kw", [dict(), dict(max_elems_per_launch=1), dict(passes_per_launch=1)])
def test_losses_before_a_wake(torch, kw):
    """Apertures lose particles in runs that precede a wake within one call:
    the lazily compacted beam must be packed before the histogram, and runs
    after a lossy run skip the slots of the particles it lost."""
    a = dict(aperture="RECT", ax=1.5e-3, ay=1.5e-3)
    lat = [Element("EDRIFT", L=2.0, **a), Element("QUAD", L=0.2, k=1.2, **a),
           Element("RFCA", volt=20e6, phase=math.radians(-20), freq=1.3e9),
           Element("EDRIFT", L=1.0, **a),
           Element("WAKE", wake_A=1e14, wake_tau0=10e-12, wake_omega=2 * math.pi * 50e9,
                   charge=1e-9, nbins=256),
           Element("MAP2", coef=inputs.chicane_coef())]
    d = inputs.gaussian_beam(20_000, seed=8, sigmas=WIDE)
    g = run_gpu(lat, d, 3, p_ref=inputs.BC_P0_EV, wake_mode=B.WAKE_FP64, **kw)
    r = run_oracle(lat, d, 3, p_ref=inputs.BC_P0_EV)
    assert 0 < r["n_alive"] < 20_000
    assert_bit_exact(g, r)


@pytest.mark.parametrize("n", [100_000, 4_000_000])
def test_bunch_compressor_fp64_bit_exact(torch, n):
    lat = inputs.bc_lattice()
    d = inputs.gaussian_beam(n, seed=0, chirp=inputs.BC_CHIRP)
    g = run_gpu(lat, d, 1, p_ref=inputs.BC_P0_EV, wake_mode=B.WAKE_FP64)
    r = run_oracle(lat, d, 1, p_ref=inputs.BC_P0_EV)
    assert_bit_exact(g, r)


@pytest.mark.parametrize("kw", [dict(run_hist=-1), dict(max_elems_per_launch=1),
                                dict(run_ppt=2, run_blocks=3)])
def test_bunch_compressor_run_binned_histograms(torch, kw):
    """Runs of RF and wake kicks (s and the alive set unchanged) bin the next
    wake's histogram themselves over the last histogram's range; with that
    off, one element per launch (the buffer cleared by its own launch
    instead of the convolution), or a few workgroups, two passes stay
    bit-exact with the oracle."""
    lat = inputs.bc_lattice()
    d = inputs.gaussian_beam(100_000, seed=2, chirp=inputs.BC_CHIRP)
    g = run_gpu(lat, d, 2, p_ref=inputs.BC_P0_EV, wake_mode=B.WAKE_FP64, **kw)
    r = run_oracle(lat, d, 2, p_ref=inputs.BC_P0_EV)
    assert_bit_exact(g, r)


def test_run_binned_histograms_mixed_bins(torch):
    """Consecutive wakes with different bin counts (the range carries over,
    the binning does not) and a marker inside the binning run."""
    wk = dict(wake_A=1e14, wake_tau0=10e-12, wake_omega=2 * math.pi * 50e9, charge=1e-9)
    rf = dict(volt=20e6, phase=math.radians(-20), freq=1.3e9)
    lat = [Element("RFCA", **rf), Element("WAKE", nbins=256, **wk), Element("RFCA", **rf),
           Element("MARKER"), Element("WAKE", nbins=1024, **wk), Element("RFCA", **rf),
           Element("WAKE", nbins=17, **wk), Element("MAP2", coef=inputs.chicane_coef())]
    d = inputs.gaussian_beam(50_000, seed=3, chirp=inputs.BC_CHIRP)
    g = run_gpu(lat, d, 2, p_ref=inputs.BC_P0_EV, wake_mode=B.WAKE_FP64)
    r = run_oracle(lat, d, 2, p_ref=inputs.BC_P0_EV)
    assert_bit_exact(g, r)
    f32 = [run_gpu(lat, d, 2, p_ref=inputs.BC_P0_EV, wake_mode=B.WAKE_FP32_MFMA, run_hist=h)
           for h in (0, -1)]
    assert np.array_equal(f32[0]["z"], f32[1]["z"]) and np.array_equal(f32[0]["id"], f32[1]["id"])


@pytest.mark.parametrize("kw", [dict(), dict(run_ppt=2, run_blocks=5)])
def test_run_binned_histograms_at_the_bin_limits(torch, kw):
    """Run-binned histograms at the largest bin count a wake may have (the
    run's LDS sub-histogram at its maximum) and at the smallest, on a ragged
    beam: bit-exact with the oracle."""
    wk = dict(wake_A=1e14, wake_tau0=10e-12, wake_omega=2 * math.pi * 50e9, charge=1e-9)
    rf = dict(volt=20e6, phase=math.radians(-20), freq=1.3e9)
    lat = [Element("RFCA", **rf), Element("WAKE", nbins=B.MAX_BINS, **wk), Element("RFCA", **rf),
           Element("WAKE", nbins=B.MAX_BINS, **wk), Element("RFCA", **rf),
           Element("WAKE", nbins=2, **wk), Element("RFCA", **rf), Element("WAKE", nbins=2, **wk),
           Element("MAP2", coef=inputs.chicane_coef())]
    d = inputs.gaussian_beam(30_001, seed=6, chirp=inputs.BC_CHIRP)
    g = run_gpu(lat, d, 2, p_ref=inputs.BC_P0_EV, wake_mode=B.WAKE_FP64, **kw)
    r = run_oracle(lat, d, 2, p_ref=inputs.BC_P0_EV)
    assert_bit_exact(g, r)


def test_run_binned_histograms_with_random_kicks(torch):
    """A random energy kick moves neither s nor the alive set: runs holding
    one still bin the next histogram, bit-exact with the oracle (Philox)."""
    wk = dict(wake_A=1e14, wake_tau0=10e-12, wake_omega=2 * math.pi * 50e9, charge=1e-9,
              nbins=512)
    rf = dict(volt=20e6, phase=math.radians(-20), freq=1.3e9)
    lat = [Element("RFCA", **rf), Element("WAKE", **wk), Element("RADKICK", sigma=1e-4),
           Element("RFCA", **rf), Element("WAKE", **wk), Element("RADKICK", sigma=1e-4),
           Element("WAKE", **wk), Element("MAP2", coef=inputs.chicane_coef())]
    d = inputs.gaussian_beam(40_000, seed=4, chirp=inputs.BC_CHIRP)
    g = run_gpu(lat, d, 2, p_ref=inputs.BC_P0_EV, seed=11, wake_mode=B.WAKE_FP64)
    r = run_oracle(lat, d, 2, p_ref=inputs.BC_P0_EV, seed=11)
    assert_bit_exact(g, r)


@pytest.mark.parametrize("n", [100_000, 4_000_000])
def test_bunch_compressor_fp32_mfma_within_bound(torch, n):
    lat = inputs.bc_lattice()
    d = inputs.gaussian_beam(n, seed=0, chirp=inputs.BC_CHIRP)
    g = run_gpu(lat, d, 1, p_ref=inputs.BC_P0_EV, wake_mode=B.WAKE_FP32_MFMA)
    r = run_oracle(lat, d, 1, p_ref=inputs.BC_P0_EV)
    assert g["n_alive"] == r["n_alive"] == n
    assert np.array_equal(g["id"], r["id"])
    for k in (0, 1, 2, 3):
        assert np.array_equal(g["z"][k], r["z"][k])
    bd = bc_bound_on_delta(d, lat, n)
    err_d = np.abs(g["z"][5] - r["z"][5]).max()
    assert err_d <= bd, (err_d, bd)
    dmax = np.abs(r["z"][5]).max() + bd
    err_s = np.abs(g["z"][4] - r["z"][4]).max()
    assert err_s <= (0.05 + 2 * 0.075 * dmax) * bd * 1.0001 + 1e-18, (err_s, bd)
    print(f"FP32 wake: max |d delta| = {err_d:.3e} (bound {bd:.3e}), max |d s| = {err_s:.3e}")


@pytest.mark.parametrize("ppt,blocks", [(4, 2), (8, 1), (1, 3), (2, 0)])
@pytest.mark.parametrize("n", [1, 255, 4099, 30001])
def test_longitudinal_runs_ragged(torch, n, ppt, blocks):
    """The two-coordinate run path loads each thread's next particles while
    the current ones go through the elements: grids capped at a few blocks
    give several sweeps per thread and a ragged last sweep."""
    lat = inputs.bc_lattice(nbins=64)
    d = inputs.gaussian_beam(n, seed=n, chirp=inputs.BC_CHIRP)
    g = run_gpu(lat, d, 2, p_ref=inputs.BC_P0_EV, wake_mode=B.WAKE_FP64, run_ppt=ppt,
                run_blocks=blocks)
    r = run_oracle(lat, d, 2, p_ref=inputs.BC_P0_EV)
    assert_bit_exact(g, r)


# ------------------------------------------------------------------ collective calls
def test_histogram_bit_exact(torch):
    for n, nb in [(1, 8), (1000, 1024), (123457, 1024), (300000, 4096), (5000, 2)]:
        d = inputs.gaussian_beam(n, seed=n)
        beam = B.Beam.from_inputs(d)
        ws = B.Workspace(beam.n)
        rg, cnt = B.histogram(beam, nb, ws)
        rr, rc = oracle.histogram(d["z"][4], d["lost_at"], nb)
        assert np.array_equal(rg.cpu().numpy(), rr)
        assert np.array_equal(cnt.cpu().numpy().view(np.uint32), rc)


def test_histogram_nobody_alive(torch):
    d = inputs.gaussian_beam(500, seed=1)
    beam = B.Beam(d["z"], d["id"], d["lost_at"], n_alive=0)
    ws = B.Workspace(beam.n)
    rg, cnt = B.histogram(beam, 64, ws)
    assert rg.cpu().numpy().tolist() == [0.0, 0.0] and int(cnt.sum()) == 0


@pytest.mark.parametrize("nb", [2, 17, 1024, 4096])
def test_convolution(torch, nb):
    rng = np.random.default_rng(nb)
    cnt = rng.integers(0, 20000, nb).astype(np.uint32)
    rg = np.array([-2e-3, 3e-3])
    tau0, om = 10e-12, 2 * math.pi * 50e9
    w = oracle.wake_table(rg[0], rg[1], nb, tau0, om)
    ref = oracle.convolve(cnt, w)
    ct = torch.tensor(cnt.view(np.int32), device="cuda")
    rt = torch.tensor(rg, device="cuda")
    v64 = B.wake_convolve(ct, nb, rt, tau0, om, B.WAKE_FP64).cpu().numpy()
    assert np.array_equal(v64, ref)
    v32 = B.wake_convolve(ct, nb, rt, tau0, om, B.WAKE_FP32_MFMA).cpu().numpy()
    scale = np.convolve(cnt.astype(float), np.abs(w))[:nb]
    bound = (nb + 2) * 2.0 ** -24 * scale
    assert np.all(np.abs(v32 - ref) <= bound + 1e-300)
    print(f"nb={nb}: FP32 max rel err {np.max(np.abs(v32 - ref) / np.maximum(scale, 1e-300)):.2e}")


def test_wake_kick_call(torch):
    d = inputs.gaussian_beam(50_000, seed=5)
    nb, tau0, om, A, Q, P = 256, 10e-12, 2 * math.pi * 50e9, 1e14, 1e-9, 1e8
    beam = B.Beam.from_inputs(d)
    ws = B.Workspace(beam.n)
    rg, cnt = B.histogram(beam, nb, ws)
    B.wake_kick(beam, cnt, nb, rg, A, tau0, om, Q, P, B.WAKE_FP64, ws)
    got = beam.host()
    ref = oracle.Beam.from_inputs(d)
    rr, rc = oracle.histogram(ref.z[4], ref.lost_at, nb)
    v = oracle.convolve(rc, oracle.wake_table(rr[0], rr[1], nb, tau0, om))
    oracle.wake_kick(ref, rr, v, oracle.wake_kfac(Q, ref.n0, A, P))
    assert np.array_equal(got["z"], ref.z)


def test_moments_call(torch):
    for n in (1, 2, 1000, 300_001):
        d = inputs.gaussian_beam(n, seed=n)
        d["z"] += np.array([[1e-3], [0], [-2e-3], [0], [0.3], [1e-3]])
        beam = B.Beam.from_inputs(d)
        ws = B.Workspace(beam.n)
        g = B.moments(beam, ws).cpu().numpy()
        r = oracle.moments(oracle.Beam.from_inputs(d))
        if n == 1:
            assert g[0] == 1 and np.array_equal(g[1:7], r[1:7]) and not g[7:].any()
        else:
            moments_close(g, r, rtol=1e-13)


def test_compensated_moments_call(torch):
    """trk_moments_compensated (Kahan-compensated sums, Sec. 2.4) against the
    oracle's compensated two-pass moments: means within 2 ulp, central
    moments within 1e-15 of sigma_k sigma_l; the plain call stays within its
    1e-13 of the beam scale.
    An offset beam with a lost tail exercises n_alive and the shift."""
    for n in (1, 2, 1000, 300_001, 4_000_000):
        d = inputs.gaussian_beam(n, seed=n + 7)
        d["z"] += np.array([[1e-2], [1e-5], [-2e-3], [0], [1.5], [1e-3]])
        beam = B.Beam.from_inputs(d)
        if n > 1000:
            beam.n_alive.fill_(n - n // 9)
        ws = B.Workspace(beam.n)
        g = B.moments_compensated(beam, ws).cpu().numpy()
        h = beam.host()
        ob = oracle.Beam(h["z"], h["id"], np.where(np.arange(n) < h["n_alive"], -1, 5).astype(np.int64))
        r = oracle.moments(ob)
        if n == 1:
            assert g[0] == 1 and np.array_equal(g[1:7], r[1:7]) and not g[7:].any()
            continue
        assert g[0] == r[0]
        assert np.all(np.abs(g[1:7] - r[1:7]) <= 2 * np.spacing(np.abs(r[1:7]))), (g[1:7], r[1:7])
        moments_close(g, r, rtol=1e-15)
        moments_close(B.moments(beam, ws).cpu().numpy(), r, rtol=1e-13)


@pytest.mark.parametrize("frac", [0.0, 0.003, 0.05, 0.5, 1.0])
def test_compaction_order(torch, frac):
    rng = np.random.default_rng(int(frac * 1000) + 1)
    n = 200_003
    d = inputs.gaussian_beam(n, seed=11)
    d["id"] = rng.permutation(n).astype(np.uint32)
    sel = rng.random(n) < frac
    la = np.full(n, -1, np.int64)
    la[sel] = (rng.integers(5, 9, sel.sum()) << 32) | rng.integers(0, 401, sel.sum())
    d["lost_at"] = la
    beam = B.Beam.from_inputs(d)
    ws = B.Workspace(beam.n)
    B.compact_lost(beam, ws)
    g = beam.host()
    ref = oracle.Beam.from_inputs(d)
    nal = oracle.compact(ref)
    assert g["n_alive"] == nal
    assert np.array_equal(g["id"], ref.id)
    assert np.array_equal(g["lost_at"], ref.lost_at)
    assert np.array_equal(g["z"], ref.z)


@pytest.mark.parametrize("passes,elems,frac", [(1000, 60000, 0.3), (1 << 20, 4001, 0.2),
                                               (1, 1, 0.4)])
def test_compaction_order_wide_and_narrow_keys(torch, passes, elems, frac):
    """Loss records spanning 26 bits of dense rank (four radix passes), 33 bits
    (beyond the multi-block sort: one workgroup sorts), and a single record
    value (no pass at all), each with more than 16384 lost particles."""
    rng = np.random.default_rng(passes + elems)
    n = 150_001
    d = inputs.gaussian_beam(n, seed=12)
    d["id"] = rng.permutation(n).astype(np.uint32)
    sel = rng.random(n) < frac
    la = np.full(n, -1, np.int64)
    la[sel] = (rng.integers(0, passes, sel.sum()) << 32) | rng.integers(0, elems, sel.sum())
    if passes > 1:
        la[np.nonzero(sel)[0][:2]] = [0, ((passes - 1) << 32) | (elems - 1)]
    d["lost_at"] = la
    beam = B.Beam.from_inputs(d)
    ws = B.Workspace(beam.n)
    B.compact_lost(beam, ws)
    g = beam.host()
    ref = oracle.Beam.from_inputs(d)
    nal = oracle.compact(ref)
    assert g["n_alive"] == nal
    assert np.array_equal(g["id"], ref.id)
    assert np.array_equal(g["lost_at"], ref.lost_at)
    assert np.array_equal(g["z"], ref.z)


def test_compaction_leaves_old_lost_region(torch):
    """Particles beyond n_alive (lost earlier) are not touched."""
    n = 10_000
    d = inputs.gaussian_beam(n, seed=3)
    la = np.full(n, -1, np.int64)
    la[8000:] = 7 << 32
    la[[10, 500, 7999]] = (9 << 32) | 3
    d["lost_at"] = la
    beam = B.Beam(d["z"], d["id"], la, n_alive=8000)
    ws = B.Workspace(beam.n)
    B.compact_lost(beam, ws)
    g = beam.host()
    assert g["n_alive"] == 7997
    assert np.array_equal(g["id"][8000:], d["id"][8000:])
    assert g["id"][7997:8000].tolist() == [10, 500, 7999]


def test_host_pointer_rejected(torch):
    import ctypes as C
    d = inputs.gaussian_beam(100, seed=0)
    beam = B.Beam.from_inputs(d)
    ws = B.Workspace(beam.n)
    host = np.zeros(100)
    st = beam.struct()
    st.x = host.ctypes.data
    rc = B.lib().trk_compact_lost(C.byref(st), ws.ptr, ws.nbytes, None)
    assert rc == B.TRK_EPTR
    rc = B.lib().trk_compact_lost(C.byref(beam.struct()), ws.ptr, 16, None)
    assert rc == B.TRK_ERANGE


# ------------------------------------------------------------------ full-size, sampled
@pytest.mark.parametrize("fusion", [1, 3])
def test_fodo_1e7_streaming_sampled(torch, fusion):
    """1e7 particles of the FODO channel with short runs, the launch shape of
    the bandwidth measurement (coordinates beyond the Infinity Cache, so the
    runs stream with non-temporal accesses), 2 passes; 600 sampled particles
    re-tracked alone by the oracle."""
    lat = inputs.fodo_lattice()
    n = 10_000_000
    d = inputs.gaussian_beam(n, seed=0, sigmas=WIDE)
    g = run_gpu(lat, d, 2, max_elems_per_launch=fusion)
    assert 0 < g["n_alive"] < n
    rng = np.random.default_rng(fusion)
    pick = np.sort(rng.choice(n, 600, replace=False))
    sub = {"z": d["z"][:, pick].copy(), "id": d["id"][pick].copy(), "lost_at": d["lost_at"][pick].copy()}
    r = run_oracle(lat, sub, 2)
    where = np.empty(n, dtype=np.int64)
    where[g["id"]] = np.arange(n)
    rows = where[r["id"]]
    assert np.array_equal(g["lost_at"][rows], r["lost_at"])
    assert np.array_equal(g["z"][:, rows], r["z"])
    assert (g["lost_at"][: g["n_alive"]] < 0).all()
    assert (g["lost_at"][g["n_alive"]:] >= 0).all()


def test_ring_full_size_sampled(torch):
    """1e6 particles of the storage-ring workload, as tracked by the bench,
    for 10 turns; 600 sampled particles re-tracked alone by the oracle
    (particles are independent and the random kicks are keyed by id)."""
    lat = inputs.ring_lattice(seed=0)
    d = inputs.gaussian_beam(1_000_000, seed=0)
    g = run_gpu(lat, d, 10, seed=2024)
    rng = np.random.default_rng(0)
    pick = np.sort(rng.choice(1_000_000, 600, replace=False))
    sub = {"z": d["z"][:, pick].copy(), "id": d["id"][pick].copy(), "lost_at": d["lost_at"][pick].copy()}
    r = run_oracle(lat, sub, 10, seed=2024)
    where = {int(i): j for j, i in enumerate(g["id"])}
    rows = np.array([where[int(i)] for i in r["id"]])
    assert np.array_equal(g["lost_at"][rows], r["lost_at"])
    assert np.array_equal(g["z"][:, rows], r["z"])
    assert (g["lost_at"][: g["n_alive"]] < 0).all()


@pytest.mark.parametrize("shape", ["one", "same_s", "two_s"])
def test_bunch_compressor_degenerate_beams(torch, shape):
    """Wakes on degenerate bunches: a single particle, a bunch whose
    particles all share one s (histogram range of width zero: every count in
    bin 0, every lag zero) and a bunch on two values of s.  Binary64 wakes
    bit-exact with the oracle; FP32 matrix-core wakes within their bound."""
    n = 1 if shape == "one" else 5000
    d = inputs.gaussian_beam(n, seed=12, chirp=inputs.BC_CHIRP)
    if shape == "same_s":
        d["z"][4][:] = 2.5e-4
    elif shape == "two_s":
        d["z"][4][:] = np.where(np.arange(n) % 3 == 0, -1e-3, 7e-4)
    lat = inputs.bc_lattice()
    g = run_gpu(lat, d, 1, p_ref=inputs.BC_P0_EV, wake_mode=B.WAKE_FP64)
    r = run_oracle(lat, d, 1, p_ref=inputs.BC_P0_EV)
    assert_bit_exact(g, r)
    f = run_gpu(lat, d, 1, p_ref=inputs.BC_P0_EV, wake_mode=B.WAKE_FP32_MFMA)
    assert f["n_alive"] == r["n_alive"] == n
    for k in (0, 1, 2, 3):
        assert np.array_equal(f["z"][k], r["z"][k])
    bd = bc_bound_on_delta(d, lat, n)
    assert np.abs(f["z"][5] - r["z"][5]).max() <= bd


def test_bunch_compressor_streaming_runs(torch):
    """Non-temporal loads and stores in the two-coordinate kick runs (the
    form the runs take when s and delta exceed the Infinity Cache, as at 4e7
    particles), forced here on 100001 particles: binary64 wakes bit-exact with
    the oracle over two passes, FP32 wakes bit-identical to the cached form."""
    lat = inputs.bc_lattice()
    d = inputs.gaussian_beam(100_001, seed=14, chirp=inputs.BC_CHIRP)
    g = run_gpu(lat, d, 2, p_ref=inputs.BC_P0_EV, wake_mode=B.WAKE_FP64, run_nt=1)
    r = run_oracle(lat, d, 2, p_ref=inputs.BC_P0_EV)
    assert_bit_exact(g, r)
    f = [run_gpu(lat, d, 2, p_ref=inputs.BC_P0_EV, wake_mode=B.WAKE_FP32_MFMA, run_nt=nt)
         for nt in (1, -1)]
    assert np.array_equal(f[0]["z"], f[1]["z"]) and np.array_equal(f[0]["id"], f[1]["id"])
