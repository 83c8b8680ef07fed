"""Pins of the oracle's own elementary functions and of Philox4x32-10.

The own sin/cos/log/exp are checked against 50-digit mpmath values; the
argument reduction against sin of the binary64 neighbours of multiples of
pi/2 (whose exact values are tiny and known to high precision).  Philox is
checked against the published known-answer vectors and against torch's
independent header-only engine; Box-Muller normals against a KS test.
"""
import math
import os
import subprocess

import mpmath as mp
import numpy as np
import pytest
from scipy import stats

mp.mp.dps = 50
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ulps(got, exact):
    exact_f = float(exact)
    sp = np.spacing(abs(exact_f)) if exact_f != 0.0 else np.spacing(0.0)
    return abs(float(mp.mpf(got) - exact)) / sp


@pytest.mark.parametrize("name,dom", [("sin", (-8.0, 8.0)), ("cos", (-8.0, 8.0)),
                                      ("log", (1e-16, 1.0)), ("exp", (-40.0, 0.0))])
def test_own_functions_within_2ulp(orc, name, dom):
    f = getattr(orc, name)
    g = {"sin": mp.sin, "cos": mp.cos, "log": mp.log, "exp": mp.exp}[name]
    rng = np.random.default_rng(11)
    xs = list(rng.uniform(*dom, 1500))
    if name == "log":
        xs += list(np.exp(rng.uniform(-36.0, 0.0, 500))) + [1.0, 0.5, 2.0 ** -53, 0.75]
    worst = max(ulps(f(float(x)), g(mp.mpf(float(x)))) for x in xs)
    assert worst <= 2.0, worst


def test_own_functions_exact_points(orc):
    assert orc.sin(0.0) == 0.0 and orc.cos(0.0) == 1.0
    assert orc.log(1.0) == 0.0 and orc.exp(0.0) == 1.0
    assert orc.log(2.0) == pytest.approx(math.log(2.0), rel=2e-16)
    assert orc.exp(-800.0) == 0.0


@pytest.mark.parametrize("k", [1, 2, 3, 4, 7, 12, 100, 1001])
def test_reduction_near_multiples_of_half_pi(orc, k):
    # x = fl(k pi/2) differs from k pi/2 by ~1e-16: sin/cos there are tiny
    # and only a correct three-part reduction gets them to full precision.
    x = float(mp.mpf(k) * mp.pi / 2)
    for f, g in ((orc.sin, mp.sin), (orc.cos, mp.cos)):
        exact = g(mp.mpf(x))
        if abs(exact) < 1e-10:
            assert abs(float(mp.mpf(f(x)) - exact)) <= 4 * abs(float(exact)) * 2.0 ** -52 + 1e-300
        else:
            assert ulps(f(x), exact) <= 2.0


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[:4], v[4:6], v[6:10]))
    return rows


def test_philox_published_kat(orc):
    for ctr, key, out in _kat():
        assert orc.philox4x32_10(ctr, key) == out


@pytest.fixture(scope="module")
def torch_kat(tmp_path_factory):
    import torch.utils.cpp_extension as ce
    exe = str(tmp_path_factory.mktemp("kat") / "kat")
    src = os.path.join(GOLDEN, "philox_torch_kat.cpp")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", ce.include_paths()[0], src, "-o", exe],
                   check=True)
    return exe


def test_philox_vs_torch_engine(orc, torch_kat):
    rng = np.random.default_rng(5)
    words = rng.integers(0, 2 ** 32, size=(300, 6), dtype=np.uint64)
    words[:50, 1:4] = 0                      # small counters, as used for (id, step, tag, 0)
    inp = "\n".join(" ".join("%08x" % int(w) for w in row) for row in words) + "\n"
    out = subprocess.run([torch_kat], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [[int(t, 16) for t in ln.split()] for ln in out.strip().splitlines()]
    for row, r in zip(words, ref):
        assert orc.philox4x32_10([int(v) for v in row[:4]], [int(v) for v in row[4:]]) == r


def test_box_muller_normal(orc):
    g = np.array([orc.gauss(i, 7, 2, 0x1234_5678_9ABC) for i in range(40000)])
    assert abs(g.mean()) < 4.0 / math.sqrt(len(g))
    assert abs(g.std() - 1.0) < 4.0 * math.sqrt(0.5 / len(g))
    assert stats.kstest(g, "norm").pvalue > 1e-3
    # different steps and tags give independent streams
    h = np.array([orc.gauss(i, 8, 2, 0x1234_5678_9ABC) for i in range(40000)])
    assert abs(np.corrcoef(g, h)[0, 1]) < 4.0 / math.sqrt(len(g))


def test_yoshida_coefficients(orc):
    c, d = orc.yoshida()
    # consistency conditions of a 4th-order symmetric composition
    assert math.isclose(c.sum(), 1.0, rel_tol=0, abs_tol=4e-16)
    assert math.isclose(d.sum(), 1.0, rel_tol=0, abs_tol=4e-16)
    w1, w0 = d[0], d[1]
    assert math.isclose(2 * w1 ** 3 + w0 ** 3, 0.0, abs_tol=1e-14)
    # w1 = 1/(2 - 2^(1/3)) from the correctly rounded cube root of 2
    cr = float(mp.cbrt(2))
    assert w1 == 1.0 / (2.0 - cr) and w0 == -cr / (2.0 - cr)
