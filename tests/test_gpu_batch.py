"""Batched persistent launch: every variant's particles equal the same variant
tracked alone (bit for bit), for every launch schedule, through hipGraph
replays; one variant is also checked against the CPU oracle."""
import numpy as np
import pytest

from paper_1710_07350_amd import binding as B
from paper_1710_07350_amd import inputs

from helpers import moments_close, run_oracle

pytestmark = pytest.mark.gpu

SIG = (2.5e-3, 2.5e-4, 1.8e-3, 1.8e-4, 1e-3, 1e-3)  # wide: some losses


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def make_batch(nvar=10, lo=40, hi=3000, ncells=8):
    sizes = inputs.batch_variant_sizes(nvar, seed=1, lo=lo, hi=hi)
    sizes[0] = 1                                   # a one-particle variant
    lats = [inputs.ring_lattice(seed=100 + v, ncells=ncells) for v in range(nvar)]
    beams = [inputs.gaussian_beam(int(n), seed=1000 + v, sigmas=SIG) for v, n in enumerate(sizes)]
    seeds = np.array([7 + 13 * v for v in range(nvar)], dtype=np.uint64)
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cat = {"z": np.concatenate([b["z"] for b in beams], axis=1),
           "id": np.concatenate([b["id"] for b in beams]),
           "lost_at": np.concatenate([b["lost_at"] for b in beams])}
    return lats, beams, seeds, seg, cat


def run_batched(torch, lats, seg, seeds, cat, passes, **tune):
    Ls = [B.Lattice(l) for l in lats]
    bt = B.Batch(Ls, seg, seeds)
    beam = B.Beam.from_inputs(cat)
    ws = bt.workspace(64)
    mom = torch.zeros((len(lats), passes, 28), dtype=torch.float64, device="cuda")
    B.track_batched(bt, beam, passes, ws, moments=mom, **tune)
    torch.cuda.synchronize()
    return beam.host(), mom.cpu().numpy()


def alone(torch, lat, d, passes, seed):
    beam = B.Beam.from_inputs(d)
    ws = B.Workspace(beam.n)
    L = B.Lattice(lat)
    mom = torch.zeros((passes, 28), dtype=torch.float64, device="cuda")
    B.track(beam, L, passes, ws, seed=int(seed), moments=mom)
    torch.cuda.synchronize()
    h = beam.host()
    h["moments"] = mom.cpu().numpy()
    return h


def by_id(z, ids, lost):
    order = np.argsort(ids, kind="stable")
    return z[:, order], ids[order], lost[order]


@pytest.fixture(scope="module")
def case(torch):
    lats, beams, seeds, seg, cat = make_batch()
    passes = 12
    refs = [alone(torch, lats[v], beams[v], passes, seeds[v]) for v in range(len(lats))]
    return lats, beams, seeds, seg, cat, passes, refs


@pytest.mark.parametrize("tune", [dict(ppt=1, blocks_per_cu=2, use_graph=False),
                                  dict(ppt=2, blocks_per_cu=1, passes_per_launch=5, use_graph=True),
                                  dict(ppt=4, blocks_per_cu=4, use_graph=True)])
def test_batched_equals_variants_alone(torch, case, tune):
    lats, beams, seeds, seg, cat, passes, refs = case
    got, mom = run_batched(torch, lats, seg, seeds, cat, passes, **tune)
    for v in range(len(lats)):
        sl = slice(seg[v], seg[v + 1])
        gz, gi, gl = by_id(got["z"][:, sl], got["id"][sl], got["lost_at"][sl])
        r = refs[v]
        rz, ri, rl = by_id(r["z"], r["id"], r["lost_at"])
        assert np.array_equal(gi, ri)
        assert np.array_equal(gl, rl), v
        assert np.array_equal(gz, rz), v
        moments_close(mom[v], r["moments"], rtol=1e-11) if r["n_alive"] > 1 else None
    assert sum(int((r["lost_at"] >= 0).sum()) for r in refs) > 0      # losses exercised


def test_one_variant_against_oracle(torch, case):
    lats, beams, seeds, seg, cat, passes, refs = case
    v = 3
    r = run_oracle(lats[v], beams[v], passes, seed=int(seeds[v]))
    gz, gi, gl = by_id(refs[v]["z"], refs[v]["id"], refs[v]["lost_at"])
    oz, oi, ol = by_id(r["z"], r["id"], r["lost_at"])
    assert np.array_equal(gl, ol) and np.array_equal(gz, oz)


def test_graph_replays_match_eager(torch, case):
    """The captured sequence replayed several times, with eager work and
    synchronisations between replays, reproduces the eager result each time."""
    lats, beams, seeds, seg, cat, passes, refs = case
    Ls = [B.Lattice(l) for l in lats]
    bt = B.Batch(Ls, seg, seeds)
    beam = B.Beam.from_inputs(cat)
    init = (beam.z.clone(), beam.lost_at.clone())
    ws = bt.workspace(64)
    B.track_batched(bt, beam, 6, ws, use_graph=False)
    torch.cuda.synchronize()
    eager = beam.host()
    for rep in range(3):
        beam.z.copy_(init[0])
        beam.lost_at.copy_(init[1])
        junk = torch.randn(1000, device="cuda").sum()          # eager work between replays
        B.track_batched(bt, beam, 6, ws, use_graph=True)
        torch.cuda.synchronize()
        h = beam.host()
        assert float(junk) == float(junk)
        assert np.array_equal(h["z"], eager["z"]) and np.array_equal(h["lost_at"], eager["lost_at"]), rep


def test_batch_rejects_mismatched_structure(torch):
    a = B.Lattice(inputs.ring_lattice(seed=1, ncells=2))
    b = B.Lattice(inputs.ring_lattice(seed=2, ncells=3))
    with pytest.raises(B.TrkError):
        B.Batch([a, b], np.array([0, 10, 20]), np.array([1, 2], dtype=np.uint64))
    rf = B.Lattice(inputs.bc_lattice(ncav=1))
    with pytest.raises(B.TrkError):
        B.Batch([rf], np.array([0, 10]), np.array([1], dtype=np.uint64))


def test_batched_moments_of_offset_beams_match_the_oracle(torch):
    """Moments of variants whose beams sit far from the origin (an x offset
    of 2 mm, s offset by 1 m) and of a variant that loses every particle at
    its first element, against the oracle's compensated two-pass moments:
    within 1e-12 of the beam scale, and all zero for the empty variant."""
    nvar, passes = 4, 6
    sizes = np.array([3000, 1700, 900, 500])
    lats = [inputs.ring_lattice(seed=200 + v, ncells=8) for v in range(nvar)]
    lats[3][0].ax, lats[3][0].ay = 1e-7, 1e-7      # nobody survives the first element
    assert lats[3][0].aperture != "NONE"
    beams = [inputs.gaussian_beam(int(n), seed=2000 + v) for v, n in enumerate(sizes)]
    for b in beams[:3]:
        b["z"][0] += 2e-3
        b["z"][4] += 1.0
    seeds = np.array([11 + v for v in range(nvar)], dtype=np.uint64)
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cat = {"z": np.concatenate([b["z"] for b in beams], axis=1),
           "id": np.concatenate([b["id"] for b in beams]),
           "lost_at": np.concatenate([b["lost_at"] for b in beams])}
    for tune in (dict(ppt=1, blocks_per_cu=2, use_graph=False),
                 dict(ppt=4, blocks_per_cu=1, passes_per_launch=4, use_graph=True)):
        got, mom = run_batched(torch, lats, seg, seeds, cat, passes, **tune)
        for v in range(nvar):
            r = run_oracle(lats[v], beams[v], passes, seed=int(seeds[v]), moments=True)
            if v == 3:
                assert r["n_alive"] == 0 and (r["moments"] == 0).all()
                assert (mom[v] == 0).all()
                continue
            assert r["n_alive"] > 0
            moments_close(mom[v], r["moments"], rtol=1e-12)
            sl = slice(seg[v], seg[v + 1])
            gz, gi, gl = by_id(got["z"][:, sl], got["id"][sl], got["lost_at"][sl])
            oz, oi, ol = by_id(r["z"], r["id"], r["lost_at"])
            assert np.array_equal(gl, ol) and np.array_equal(gz, oz)


@pytest.fixture(scope="module")
def config_batch(torch):
    """The batched scan at its configured shape: 256 ring variants of 40
    cells, each with its own sextupoles (PCG64 draws, seed 100 + v), Gaussian beams of the C-FODO sigmas with log-uniform sizes in
    [1e3, 1e5], 200 turns, moments every turn, one graph-captured launch
    sequence."""
    nvar, turns = 256, 200
    sizes = inputs.batch_variant_sizes(nvar, seed=0)
    lats = [inputs.ring_lattice(seed=100 + v) for v in range(nvar)]
    beams = [inputs.gaussian_beam(int(n), seed=1000 + v) for v, n in enumerate(sizes)]
    seeds = np.array([7 + 13 * v for v in range(nvar)], dtype=np.uint64)
    seg = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    cat = {"z": np.concatenate([b["z"] for b in beams], axis=1),
           "id": np.concatenate([b["id"] for b in beams]),
           "lost_at": np.concatenate([b["lost_at"] for b in beams])}
    got, mom = run_batched(torch, lats, seg, seeds, cat, turns, ppt=1, blocks_per_cu=8,
                           use_graph=True)
    return sizes, lats, beams, seeds, seg, got, mom, turns


def test_config_batch_against_the_oracle(torch, config_batch):
    """Batched output compared with the oracle directly: for 12 variants
    (the three smallest whole, with their moments every turn; nine others on
    48-particle id subsets, particles being independent and their kicks keyed
    by id), coordinates and loss records bit-exact after 200 turns."""
    sizes, lats, beams, seeds, seg, got, mom, turns = config_batch
    assert seg[-1] > 4_000_000
    rng = np.random.default_rng(5)
    small = np.argsort(sizes)[:3]
    others = rng.choice(np.setdiff1d(np.arange(len(sizes)), small), 9, replace=False)
    lost_total = 0
    for v in list(small) + list(others):
        sl = slice(seg[v], seg[v + 1])
        gz, gi, gl = by_id(got["z"][:, sl], got["id"][sl], got["lost_at"][sl])
        if v in small:
            d = beams[v]
        else:
            pick = np.sort(rng.choice(int(sizes[v]), 48, replace=False))
            d = {"z": beams[v]["z"][:, pick], "id": beams[v]["id"][pick],
                 "lost_at": beams[v]["lost_at"][pick]}
            gz, gi, gl = gz[:, pick], gi[pick], gl[pick]
        r = run_oracle(lats[v], d, turns, seed=int(seeds[v]), moments=v in small)
        oz, oi, ol = by_id(r["z"], r["id"], r["lost_at"])
        assert np.array_equal(gi, oi)
        assert np.array_equal(gl, ol), v
        assert np.array_equal(gz, oz), v
        if v in small:
            moments_close(mom[v], r["moments"], rtol=1e-12)
        lost_total += int((ol >= 0).sum())
    assert lost_total > 0                                   # losses exercised


def test_config_batch_every_variant_matches_its_lone_run(torch, config_batch):
    """Each of 16 variants of the configured scan tracked alone with
    trk_track (its own handle, same seed) equals its batched segment."""
    sizes, lats, beams, seeds, seg, got, mom, turns = config_batch
    for v in np.linspace(0, len(sizes) - 1, 16).astype(int):
        r = alone(torch, lats[v], beams[v], turns, seeds[v])
        sl = slice(seg[v], seg[v + 1])
        gz, gi, gl = by_id(got["z"][:, sl], got["id"][sl], got["lost_at"][sl])
        rz, ri, rl = by_id(r["z"], r["id"], r["lost_at"])
        assert np.array_equal(gl, rl) and np.array_equal(gz, rz), v
        moments_close(mom[v], r["moments"], rtol=1e-11)
