"""The allocation-free moments entry point (trk_moments_noalloc) against
trk_moments through the C-ABI: two calls in a row on one device, the second
on a smaller beam, each bit for bit equal to the workspace version (same
kernels, grid and summation order)."""
import numpy as np
import pytest

from paper_1710_07350_amd import binding as B
from paper_1710_07350_amd import inputs

pytestmark = pytest.mark.gpu


def _beam(n, seed, lost_every=0):
    d = inputs.gaussian_beam(n, seed=seed)
    d["z"][0] += 1e-2          # an offset beam: the shifted second pass matters
    b = B.Beam.from_inputs(d)
    if lost_every:
        # only a prefix is alive: the reduction must stop at n_alive
        b.n_alive.fill_(n - n // lost_every)
    return b


def test_noalloc_moments_match_workspace_moments():
    import torch
    assert torch.cuda.is_available()
    for n, seed, lost in ((300_000, 3, 7), (12_345, 4, 0)):
        beam = _beam(n, seed, lost)
        want = B.moments(beam, B.Workspace(n)).cpu().numpy()
        out = torch.full((28,), float("nan"), dtype=torch.float64, device="cuda")
        got = B.moments_noalloc(beam, out).cpu().numpy()
        assert np.array_equal(got.view(np.int64), want.view(np.int64)), (n, got, want)
        assert got[0] == float(beam.n_alive.item())


def test_noalloc_moments_empty_and_after_other_calls():
    import torch
    beam = _beam(1000, 5)
    beam.n_alive.fill_(0)
    out = torch.full((28,), float("nan"), dtype=torch.float64, device="cuda")
    got = B.moments_noalloc(beam, out).cpu().numpy()
    assert np.array_equal(got, np.zeros(28))
    # a larger beam again after the empty one: the scratch keeps no state
    beam = _beam(70_000, 6)
    want = B.moments(beam, B.Workspace(70_000)).cpu().numpy()
    got = B.moments_noalloc(beam, out).cpu().numpy()
    assert np.array_equal(got.view(np.int64), want.view(np.int64))
