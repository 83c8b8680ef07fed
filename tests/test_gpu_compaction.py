"""Parity of the paper's two loss reorderings on the GPU (sort by key and the
sparse swap) with their oracle, bit for bit, at the loss fractions of the
paper's comparison (0.5, 5, 10, 50 %) and at the edges."""
import numpy as np
import pytest

import oracle
from oracle import compaction
from paper_1710_07350_amd import binding as B
from paper_1710_07350_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def lossy(n, frac, seed, extra):
    rng = np.random.default_rng(seed)
    d = inputs.gaussian_beam(n + extra, seed=seed)
    d["id"] = rng.permutation(n + extra).astype(np.uint32)
    la = np.full(n + extra, -1, np.int64)
    sel = rng.random(n) < frac
    la[:n][sel] = (rng.integers(0, 9, sel.sum()) << 32) | rng.integers(0, 401, sel.sum())
    la[n:] = (77 << 32) | 5                      # older losses beyond n_alive
    d["lost_at"] = la
    return d


@pytest.mark.parametrize("mode", [B.COMPACT_SWAP, B.COMPACT_SORT])
@pytest.mark.parametrize("n,frac,extra", [(200_003, 0.005, 0), (200_003, 0.05, 17),
                                          (200_003, 0.1, 0), (200_003, 0.5, 1000),
                                          (4099, 1.0, 3), (4099, 0.0, 0), (1, 1.0, 0),
                                          (257, 0.3, 256)])
def test_compaction_variant_bit_exact(torch, mode, n, frac, extra):
    d = lossy(n, frac, n + int(frac * 1000), extra)
    beam = B.Beam(d["z"], d["id"], d["lost_at"], n_alive=n)
    ws = B.Workspace(beam.n)
    B.compact_lost(beam, ws, mode=mode)
    g = beam.host()
    ref = oracle.Beam.from_inputs(d)
    fn = compaction.compact_swap if mode == B.COMPACT_SWAP else compaction.compact_sort
    nal = fn(ref, n)
    assert g["n_alive"] == nal
    assert np.array_equal(g["id"], ref.id)
    assert np.array_equal(g["lost_at"], ref.lost_at)
    assert np.array_equal(g["z"], ref.z)


def test_compaction_variants_repeat_on_a_compacted_beam(torch):
    """A second call with nothing newly lost changes nothing."""
    d = lossy(50_000, 0.1, 3, 0)
    for mode in (B.COMPACT_SWAP, B.COMPACT_SORT):
        beam = B.Beam(d["z"], d["id"], d["lost_at"], n_alive=50_000)
        ws = B.Workspace(beam.n)
        B.compact_lost(beam, ws, mode=mode)
        once = beam.host()
        B.compact_lost(beam, ws, mode=mode)
        twice = beam.host()
        for k in ("z", "id", "lost_at", "n_alive"):
            assert np.array_equal(once[k], twice[k])


@pytest.mark.parametrize("mode", [B.COMPACT_STABLE, B.COMPACT_SWAP, B.COMPACT_SORT])
def test_alive_count_above_the_beam_counts_as_the_beam(torch, mode):
    """*n_alive beyond n_total acts as n_total (no slot past the arrays is
    read) and the clamped count minus the losses is stored back."""
    n = 4096 * 3 + 100                           # ragged last tile
    d = lossy(n, 0.05, 11, 0)
    over = B.Beam(d["z"], d["id"], d["lost_at"], n_alive=n + 5000)
    exact = B.Beam(d["z"], d["id"], d["lost_at"], n_alive=n)
    for b in (over, exact):
        B.compact_lost(b, B.Workspace(b.n), mode=mode)
    g, e = over.host(), exact.host()
    assert g["n_alive"] == e["n_alive"] < n
    for k in ("z", "id", "lost_at"):
        assert np.array_equal(g[k], e[k])
