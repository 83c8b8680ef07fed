"""Pins of the oracle's two alternatives to the stable loss reordering: the
paper's sort by key and its sparse swap (Sec. 2.5), by invariants that any
slip in the index bookkeeping breaks."""
import numpy as np
import pytest

from oracle import compaction


def make(orc, n, frac, seed, extra=0):
    rng = np.random.default_rng(seed)
    z = rng.normal(0, 1, (6, n + extra))
    la = np.full(n + extra, -1, np.int64)
    lost = rng.random(n) < frac
    la[:n][lost] = (rng.integers(0, 5, lost.sum()) << 32) | rng.integers(0, 60, lost.sum())
    la[n:] = 99 << 32                       # older losses beyond n_alive
    return orc.Beam(z, np.arange(n + extra, dtype=np.uint32), la)


def snapshot(b):
    return b.z.copy(), b.id.copy(), b.lost_at.copy()


@pytest.mark.parametrize("n,frac", [(20, 0.2), (1000, 0.005), (1000, 0.05), (997, 0.1),
                                    (5000, 0.5), (300, 0.0), (64, 1.0)])
def test_sort_by_key_is_a_stable_partition(orc, n, frac):
    b = make(orc, n, frac, n, extra=7)
    z0, id0, la0 = snapshot(b)
    m = compaction.compact_sort(b, n)
    alive = np.nonzero(la0[:n] < 0)[0]
    lost = np.nonzero(la0[:n] >= 0)[0]
    assert m == len(alive)
    order = np.concatenate([alive, lost])
    assert np.array_equal(b.id[:n], id0[order])
    assert np.array_equal(b.z[:, :n], z0[:, order]) and np.array_equal(b.lost_at[:n], la0[order])
    assert np.array_equal(b.id[n:], id0[n:]) and np.array_equal(b.z[:, n:], z0[:, n:])


@pytest.mark.parametrize("n,frac", [(20, 0.2), (1000, 0.005), (1000, 0.05), (997, 0.1),
                                    (5000, 0.5), (300, 0.0), (64, 1.0), (2, 0.5)])
def test_sparse_swap_invariants(orc, n, frac):
    b = make(orc, n, frac, 10 + n, extra=5)
    z0, id0, la0 = snapshot(b)
    m = compaction.compact_swap(b, n)
    alive0 = la0[:n] < 0
    assert m == alive0.sum()
    # a permutation of the first n slots carrying whole particles
    pos = {int(i): j for j, i in enumerate(id0)}
    src = np.array([pos[int(i)] for i in b.id[:n]])
    assert sorted(src.tolist()) == list(range(n))
    assert np.array_equal(b.z[:, :n], z0[:, src]) and np.array_equal(b.lost_at[:n], la0[src])
    # survivors fill the head, lost particles the tail
    assert (b.lost_at[:m] < 0).all() and (b.lost_at[m:n] >= 0).all()
    # sparsity: survivors already in the head and lost particles already in
    # the tail stay where they were; every other particle swaps with one
    stay = (alive0 & (np.arange(n) < m)) | (~alive0 & (np.arange(n) >= m))
    assert np.array_equal(src[stay], np.nonzero(stay)[0])
    moved = np.nonzero(~stay)[0]
    assert np.array_equal(src[src[moved]], moved)          # pairwise swaps
    holes = moved[moved < m]
    donors = moved[moved >= m]
    assert len(holes) == len(donors)
    assert np.array_equal(src[holes], donors)              # k-th hole <- k-th tail survivor
    # the older losses beyond n_alive are untouched
    assert np.array_equal(b.id[n:], id0[n:])


def test_twenty_particles_four_lost(orc):
    """The size of the paper's illustration: 20 particles, four lost, here
    three of them in the head (holes) and one already in the tail."""
    z = np.arange(120, dtype=float).reshape(6, 20)
    la = np.full(20, -1, np.int64)
    la[[1, 5, 15, 18]] = 3
    b = orc.Beam(z, np.arange(20, dtype=np.uint32), la)
    assert compaction.compact_swap(b, 20) == 16
    assert b.id.tolist() == [0, 16, 2, 3, 4, 17, 6, 7, 8, 9, 10, 11, 12, 13, 14, 19,
                             1, 5, 18, 15]
