"""Parity of third-order maps (the M3 matrix tracking) on the GPU with the
oracle: the thick-quadrupole pattern and arbitrary MAP3 elements are
bit-exact, at every fusion depth, inside tracking with losses."""
import numpy as np
import pytest

from paper_1710_07350_amd import binding as B
from paper_1710_07350_amd import inputs
from paper_1710_07350_amd.inputs import Element

from helpers import assert_bit_exact, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

WIDE = (2e-3, 2e-4, 2e-3, 2e-4, 1e-3, 1e-2)   # loses particles; delta wide for the cubic terms


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("kw", [dict(), dict(max_elems_per_launch=1), dict(passes_per_launch=3),
                                dict(max_elems_per_launch=2, run_nt=1)])
def test_fodo_third_order_quads_bit_exact(torch, kw):
    lat = inputs.fodo_lattice(quad_order=3)
    d = inputs.gaussian_beam(5000, seed=21, sigmas=WIDE)
    g = run_gpu(lat, d, 20, moments=True, **kw)
    r = run_oracle(lat, d, 20, moments=True)
    assert 0 < r["n_alive"] < 5000
    assert_bit_exact(g, r)
    # the cubic terms act: second-order quads give other coordinates
    r2 = run_oracle(inputs.fodo_lattice(), d, 20)
    assert not np.array_equal(r["z"], r2["z"])


@pytest.mark.parametrize("n", [1, 255, 4099])
def test_arbitrary_map3_bit_exact(torch, n):
    """A dense random third-order map (the generic evaluator) between drifts,
    with an aperture, over several passes."""
    rng = np.random.default_rng(n)
    coef = np.zeros(504)
    for i in range(6):
        coef[6 + 7 * i] = 1.0
    coef[6:42] += rng.normal(0, 0.05, 36)
    coef[42:168] = rng.normal(0, 0.5, 126) * (rng.random(126) < 0.5)
    coef[168:] = rng.normal(0, 2.0, 336) * (rng.random(336) < 0.5)
    coef[:6] = rng.normal(0, 1e-5, 6)
    a = dict(aperture="ELLIPSE", ax=6e-3, ay=4e-3)
    lat = [Element("EDRIFT", L=0.5, **a), Element("MAP3", coef=coef, **a),
           Element("QUAD", L=0.3, k=-0.9, order=3), Element("EDRIFT", L=0.5)]
    d = inputs.gaussian_beam(n, seed=n, sigmas=WIDE)
    for kw in (dict(), dict(max_elems_per_launch=1)):
        g = run_gpu(lat, d, 6, **kw)
        r = run_oracle(lat, d, 6)
        assert_bit_exact(g, r)


def test_map3_coefficient_count_checked(torch):
    with pytest.raises(ValueError):
        B.Lattice([Element("MAP3", coef=np.zeros(168))])


def test_fodo_third_order_1e7_sampled(torch):
    """1e7 particles through the third-order FODO channel, 2 passes, as the
    bench launches them; 500 sampled particles re-tracked by the oracle."""
    lat = inputs.fodo_lattice(quad_order=3)
    n = 10_000_000
    d = inputs.gaussian_beam(n, seed=3, sigmas=WIDE)
    g = run_gpu(lat, d, 2)
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(n, 500, replace=False))
    sub = {"z": d["z"][:, pick].copy(), "id": d["id"][pick].copy(), "lost_at": d["lost_at"][pick].copy()}
    r = run_oracle(lat, sub, 2)
    where = np.empty(n, dtype=np.int64)
    where[g["id"]] = np.arange(n)
    rows = where[r["id"]]
    assert np.array_equal(g["lost_at"][rows], r["lost_at"])
    assert np.array_equal(g["z"][:, rows], r["z"])
