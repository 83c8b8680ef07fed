"""Device arithmetic the kernels rely on, bit for bit against the CPU:
binary64 sqrt and division (correctly rounded), the own sin/cos/log/exp,
Philox4x32-10 and the Box-Muller normal."""
import numpy as np
import pytest

import oracle
from paper_1710_07350_amd import binding as B

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def test_sqrt_and_division_correctly_rounded(torch):
    rng = np.random.default_rng(0)
    n = 1 << 20
    x = np.concatenate([np.exp(rng.uniform(-700, 700, n // 2)),
                        rng.uniform(0, 2, n // 2 - 6), [0.0, 1.0, 4.0, 2.0 ** -1074, 1e-310, 1e300]])
    y = np.exp(rng.uniform(-300, 300, n)) * rng.choice([-1.0, 1.0], n)
    xt = torch.tensor(x, device="cuda")
    yt = torch.tensor(y, device="cuda")
    s = B.elementary(4, xt).cpu().numpy()
    q = B.elementary(5, xt, yt).cpu().numpy()
    assert np.array_equal(s.view(np.int64), np.sqrt(x).view(np.int64))
    assert np.array_equal(q.view(np.int64), (x / y).view(np.int64))


def test_sqrt_and_division_correctly_rounded_2e8(torch):
    """2e8 operand pairs, in chunks of 1e7: random bit patterns of finite
    binary64 values over the whole range (subnormals included), and the
    operand ranges the element kernels divide and take roots in (pz near 1,
    path lengths, slope squares).  Every quotient and root is compared bit
    for bit with the CPU's IEEE operations."""
    rng = np.random.default_rng(1)
    m = 10_000_000
    top = np.int64(0x7FEFFFFFFFFFFFFF)          # largest finite
    for chunk in range(20):
        if chunk % 2 == 0:
            bits = rng.integers(0, top, m, dtype=np.int64, endpoint=True)
            x = bits.view(np.float64) * rng.choice([-1.0, 1.0], m)
            y = rng.integers(1, top, m, dtype=np.int64, endpoint=True).view(np.float64)
            r = np.abs(x)
        else:
            x = rng.uniform(-2.0, 2.0, m)
            y = 1.0 + rng.uniform(-0.1, 0.1, m)
            r = 1.0 - rng.uniform(0.0, 1e-4, m)
        q = B.elementary(5, torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda"))
        sq = B.elementary(4, torch.tensor(r, device="cuda"))
        with np.errstate(over="ignore", under="ignore"):
            ref_q = x / y
        assert np.array_equal(q.cpu().numpy().view(np.int64), ref_q.view(np.int64)), chunk
        assert np.array_equal(sq.cpu().numpy().view(np.int64), np.sqrt(r).view(np.int64)), chunk


@pytest.mark.parametrize("fn,dom", [(0, (-9.0, 9.0)), (1, (-9.0, 9.0)), (2, (1e-300, 1.0)),
                                    (3, (-720.0, 5.0))])
def test_own_functions_bit_equal_to_oracle(torch, fn, dom):
    rng = np.random.default_rng(fn)
    if fn == 2:
        x = np.exp(rng.uniform(np.log(dom[0]), 0.0, 20000))
    else:
        x = rng.uniform(*dom, 20000)
    f = [oracle.sin, oracle.cos, oracle.log, oracle.exp][fn]
    ref = np.array([f(float(v)) for v in x])
    got = B.elementary(fn, torch.tensor(x, device="cuda")).cpu().numpy()
    assert np.array_equal(got.view(np.int64), ref.view(np.int64))


def test_philox_bit_equal(torch):
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2 ** 32, (5000, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2 ** 32, (5000, 2), dtype=np.uint64).astype(np.uint32)
    ctr[:100, 1:] = 0
    got = B.philox(torch.tensor(ctr.view(np.int32), device="cuda"),
                   torch.tensor(key.view(np.int32), device="cuda")).cpu().numpy().view(np.uint32)
    for i in range(0, 5000, 7):
        assert list(got[i]) == oracle.philox4x32_10(ctr[i].tolist(), key[i].tolist())


def test_gauss_bit_equal(torch):
    ids = np.arange(0, 300000, 37, dtype=np.uint32)
    seed = 0xDEADBEEF12345
    got = B.gauss(torch.tensor(ids.view(np.int32), device="cuda"), 17, 2, seed).cpu().numpy()
    ref = np.array([oracle.gauss(int(i), 17, 2, seed) for i in ids])
    assert np.array_equal(got.view(np.int64), ref.view(np.int64))


def test_machine_probes(torch):
    """The ceiling probes compute what they claim (their timing is the
    peak-probe script's business)."""
    n = 100_003
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for mode in (0, 2):
        dst.zero_()
        B.probe_stream(src, dst, mode, 7)
        assert torch.equal(dst, src + 1.0)
    part = torch.zeros(7, dtype=torch.float64, device="cuda")
    B.probe_stream(src, part, 1, 7)
    assert float(part.sum()) == n * (n - 1) / 2
    out = torch.empty(3 * 256, dtype=torch.float64, device="cuda")
    B.probe_fma(out, 10, 3)
    a = 1.0 + 1e-3 * np.add.outer(np.arange(256), np.arange(8))
    for _ in range(10):
        a = a * 0.999999 + 1e-7
    assert np.allclose(out.cpu().numpy()[:256], a.sum(axis=1), rtol=1e-14)
