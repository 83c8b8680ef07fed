"""Oracle of the paper's two alternatives to the stable loss reordering
(TEST INFRASTRUCTURE, like the rest of this package).

Sec. 2.5 of the paper describes, for a beam whose kernels have flagged lost
particles, a straightforward sort of the particle array by the key
  index (alive) or index + N (lost),
and the faster sparse algorithm it uses instead: sum the alive flags (skip
everything when nobody was lost); sort the keys of the tail -- the last
(number lost) slots -- so that the tail's survivors come first; scan the lost
flags of the head to number its holes; swap the k-th hole of the head with
the k-th survivor of the tail; shorten the particle count.  Survivors do not
keep their order in the second algorithm.

Both act on the slots below n_alive, whose lost particles carry a loss
record >= 0; slots beyond n_alive (older losses) are not touched.  The beam
arrays are updated in place; the new n_alive is returned.
"""
from __future__ import annotations

import numpy as np


def _move(beam, order, n):
    """Permute the first n slots of every beam array: slot j <- slot order[j]."""
    beam.z[:, :n] = beam.z[:, order]
    beam.id[:n] = beam.id[order]
    beam.lost_at[:n] = beam.lost_at[order]


def compact_sort(beam, n_alive: int) -> int:
    """Sort by key: key = i for a survivor, i + N for a lost particle."""
    n = int(n_alive)
    idx = np.arange(n, dtype=np.int64)
    lost = beam.lost_at[:n] >= 0
    key = np.where(lost, idx + n, idx)
    order = np.argsort(key, kind="stable")
    _move(beam, order, n)
    return n - int(lost.sum())


def compact_swap(beam, n_alive: int) -> int:
    """The paper's sparse swap: only holes in the head and survivors in the
    tail move."""
    n = int(n_alive)
    ret = (beam.lost_at[:n] < 0).astype(np.int64)      # 1 alive, 0 lost
    n_new = int(ret.sum())                              # sum reduction
    if n_new == n:
        return n
    idx = np.arange(n, dtype=np.int64)
    key = np.where(ret == 1, idx, idx + n)
    tail = np.sort(key[n_new:])                         # sort the tail's keys
    donors = tail[tail < n]                             # its survivors, ascending
    lost_flag = 1 - ret[:n_new]                         # 1 where the head has a hole
    scan = np.cumsum(lost_flag)                         # inclusive scan
    # where consecutive scan values differ the slot holds the scan-th hole
    is_hole = np.diff(np.concatenate([[0], scan])) != 0
    holes = np.empty(int(scan[-1]) if n_new > 0 else 0, dtype=np.int64)
    holes[scan[is_hole] - 1] = idx[:n_new][is_hole]     # the loss map
    assert len(holes) == len(donors)
    order = idx.copy()
    order[holes] = donors
    order[donors] = holes
    _move(beam, order, n)
    return n_new
