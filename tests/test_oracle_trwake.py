"""Pins of the oracle's transverse wake (the TRWAKE element): the fixed-point
dipole sums per bin, the sine resonator table, the binary64 convolution and
the kick of the canonical transverse momenta, against exact rational
arithmetic, high-precision closed forms, symmetry and causality."""
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
from scipy.signal import fftconvolve

from paper_1710_07350_amd import inputs
from paper_1710_07350_amd.inputs import Element

mp.mp.dps = 40
Q40 = 2 ** 40


def brute_quantum(x: float) -> int:
    if math.isnan(x):
        return 0
    x = min(max(x, -1.0), 1.0)
    return round(Fraction(x) * Q40)          # Fraction rounds half to even


def wrap64(v: int) -> int:
    return ((v + 2 ** 63) % 2 ** 64) - 2 ** 63


def brute_bins(s, alive, nb):
    smin, smax = Fraction(float(s[alive].min())), Fraction(float(s[alive].max()))
    out = np.full(len(s), -1, np.int64)
    for i in np.nonzero(alive)[0]:
        b = math.floor((Fraction(float(s[i])) - smin) * nb / (smax - smin))
        out[i] = min(b, nb - 1)
    return out


# ------------------------------------------------------------------ dipole sums
def test_dipole_quantum_rounding_clamp_nan(orc):
    rng = np.random.default_rng(0)
    xs = list(rng.uniform(-1.5, 1.5, 2000)) + list(rng.normal(0, 1e-3, 2000))
    ties = [(k + 0.5) / Q40 for k in range(-6, 6)]          # exact halves: to even
    xs += ties + [1.0, -1.0, 2.0, -3.0, math.inf, -math.inf, 0.0, -0.0, 5e-324]
    for x in xs:
        assert orc.dipole_quantum(x) == brute_quantum(x), x
    assert orc.dipole_quantum(math.nan) == 0
    assert [orc.dipole_quantum(t) for t in ties[:4]] == [-6, -4, -4, -2]


def test_dipole_histogram_brute_force(orc):
    rng = np.random.default_rng(1)
    n, nb = 6000, 64
    s = rng.normal(0, 1e-3, n)
    x = rng.normal(2e-4, 1e-3, n)
    y = rng.normal(-1e-4, 5e-4, n)
    x[::97] = 1.7                            # clamped
    y[::89] = np.nan                         # counts 0
    lost = np.full(n, -1, np.int64)
    lost[::5] = 3
    rg, cnt, dx, dy = orc.dipole_histogram(s, x, y, lost, nb)
    rg0, cnt0 = orc.histogram(s, lost, nb)
    assert np.array_equal(rg, rg0) and np.array_equal(cnt, cnt0)
    bins = brute_bins(s, lost < 0, nb)
    ref_x = [0] * nb
    ref_y = [0] * nb
    for i in range(n):
        if bins[i] >= 0:
            ref_x[bins[i]] += brute_quantum(float(x[i]))
            ref_y[bins[i]] += brute_quantum(float(y[i]))
    assert dx.tolist() == [wrap64(v) for v in ref_x]
    assert dy.tolist() == [wrap64(v) for v in ref_y]
    assert np.array_equal(np.bincount(bins[bins >= 0], minlength=nb), cnt)


def test_dipole_sums_are_within_half_a_quantum_per_particle_of_the_plain_sum(orc):
    """Each bin's fixed-point sum, read in metres, differs from the exact sum
    of its particles' raw x (and y) by at most half a quantum (2^-41 m) per
    particle, plus what the clamp to [-1, 1] m removes; non-finite
    coordinates count 0.  The reference is exact rational arithmetic on the
    raw coordinates (math.fsum gives the same to one rounding)."""
    rng = np.random.default_rng(7)
    n, nb = 20000, 128
    s = rng.normal(0, 1e-3, n)
    x = rng.normal(3e-4, 2e-3, n) * np.exp(rng.uniform(-8, 0, n))
    y = rng.standard_t(3, n) * 1e-3
    x[::211] = rng.uniform(1.0, 5.0, x[::211].size) * rng.choice([-1, 1], x[::211].size)
    y[::307] = np.nan
    lost = np.full(n, -1, np.int64)
    lost[::7] = 2
    rg, cnt, dx, dy = orc.dipole_histogram(s, x, y, lost, nb)
    bins = brute_bins(s, lost < 0, nb)
    for row, coord in ((dx, x), (dy, y)):
        for b in range(nb):
            sel = coord[bins == b]
            fin = sel[np.isfinite(sel)]
            exact = sum((Fraction(float(v)) for v in fin), Fraction(0))
            clamp = sum((Fraction(abs(float(v))) - 1 for v in fin if abs(v) > 1.0), Fraction(0))
            got = Fraction(int(row[b]), Q40)
            err = abs(got - exact)
            assert err <= Fraction(len(fin), 2 * Q40) + clamp, (b, float(err))
            if clamp == 0 and len(fin):
                assert abs(float(got) - math.fsum(fin)) <= len(fin) * 2.0 ** -41 + 1e-300
    # the bins together hold the whole (clamped) sum
    al = (lost < 0) & np.isfinite(x)
    tot = Fraction(sum(int(v) for v in dx), Q40)
    ref = sum((Fraction(float(v)) for v in np.clip(x[al], -1.0, 1.0)), Fraction(0))
    assert abs(tot - ref) <= Fraction(int(al.sum()), 2 * Q40)


def test_dipole_sums_are_modulo_2_64(orc):
    """2^23 particles at x = +1 m overflow the running sum, one at x = -1 m
    brings the total back into range: the modular sum is still exact."""
    n = 2 ** 23 + 1
    s = np.zeros(n)
    x = np.ones(n)
    x[-1] = -1.0
    rg, cnt, dx, dy = orc.dipole_histogram(s, x, np.zeros(n), np.full(n, -1, np.int64), 4)
    assert cnt[0] == n and dx[0] == 2 ** 63 - 2 ** 40 and dy[0] == 0


def test_dipole_mirror_beam_cancels_and_offset_scales(orc):
    rng = np.random.default_rng(2)
    s = rng.normal(0, 1e-3, 3000)
    x = rng.normal(0, 1e-3, 3000)
    ss, xx = np.concatenate([s, s]), np.concatenate([x, -x])
    lost = np.full(6000, -1, np.int64)
    rg, cnt, dx, dy = orc.dipole_histogram(ss, xx, xx, lost, 128)
    assert not dx.any() and not dy.any() and cnt.sum() == 6000
    c = 3.3e-4
    rg, cnt, dx, dy = orc.dipole_histogram(s, np.full(3000, c), np.full(3000, -c),
                                           lost[:3000], 128)
    q = brute_quantum(c)
    assert np.array_equal(dx, cnt.astype(np.int64) * q)
    assert np.array_equal(dy, -cnt.astype(np.int64) * q)
    m = orc.dipole_metres(dx)
    assert np.array_equal(m, cnt * (q / Q40))


# ------------------------------------------------------------------ table and convolution
def test_trwake_table_closed_form(orc):
    nb, smin, smax, tau0, om = 1024, -3e-3, 5e-3, 10e-12, 2 * math.pi * 50e9
    w = orc.trwake_table(smin, smax, nb, tau0, om)
    assert w[0] == 0.0
    dt = ((smax - smin) / nb) / 299792458.0
    for m in range(1, nb, 11):
        t = mp.mpf(m) * mp.mpf(dt)
        exact = mp.exp(-t / tau0) * mp.sin(om * t)
        assert abs(float(exact) - w[m]) < 2e-15
    assert not orc.trwake_table(0.0, 0.0, 16, tau0, om).any()   # zero range: no lag


@pytest.mark.parametrize("nb", [4, 9, 16])
def test_convolve_f64_exact_rational(orc, nb):
    rng = np.random.default_rng(nb)
    c = rng.normal(0, 1e-2, nb)
    w = rng.normal(0, 1, nb)
    v = orc.convolve_f64(c, w)
    for i in range(nb):
        exact = sum(Fraction(c[j]) * Fraction(w[i - j]) for j in range(i + 1))
        bound = (i + 1) * 2.0 ** -53 * sum(abs(c[j] * w[i - j]) for j in range(i + 1))
        assert abs(float(Fraction(v[i]) - exact)) <= bound


def test_convolve_f64_delta_and_fft(orc):
    nb = 1024
    w = orc.trwake_table(0.0, 8e-3, nb, 10e-12, 2 * math.pi * 50e9)
    c = np.zeros(nb)
    c[41] = 1.25e-3
    v = orc.convolve_f64(c, w)
    assert np.array_equal(v[41:], 1.25e-3 * w[:nb - 41]) and not v[:41].any()
    rng = np.random.default_rng(3)
    c = rng.normal(0, 1e-2, nb)
    v = orc.convolve_f64(c, w)
    ref = fftconvolve(c, w)[:nb]
    scale = np.convolve(np.abs(c), np.abs(w))[:nb]
    assert np.all(np.abs(v - ref) <= 1e-12 * scale.max())


# ------------------------------------------------------------------ kick
def canonical(xp, yp, dp):
    xp, yp, opd = mp.mpf(float(xp)), mp.mpf(float(yp)), 1 + mp.mpf(float(dp))
    r = mp.sqrt(1 + xp * xp + yp * yp)
    return opd * xp / r, opd * yp / r


def test_trwake_kick_adds_canonical_momentum(orc):
    """The kick adds kfac V(s) to the canonical momenta: checked by converting
    the slopes before and after to canonical momenta in 40-digit arithmetic,
    with V interpolated between bin centres by numpy (held at the ends)."""
    rng = np.random.default_rng(5)
    n, nb = 400, 32
    z = rng.normal(0, 1e-3, (6, n))
    z[1] *= 0.3
    z[3] *= 0.3
    rg = np.array([z[4].min(), z[4].max()])
    vx, vy = rng.normal(0, 1, nb), rng.normal(0, 1, nb)
    kfac = 2e-6
    b = orc.Beam(z, np.arange(n, dtype=np.uint32), np.full(n, -1, np.int64))
    orc.trwake_kick(b, rg, vx, vy, kfac)
    for k in (0, 2, 4, 5):
        assert np.array_equal(b.z[k], z[k])
    cen = rg[0] + (np.arange(nb) + 0.5) * (rg[1] - rg[0]) / nb
    ux, uy = np.interp(z[4], cen, vx), np.interp(z[4], cen, vy)
    for i in range(n):
        p0 = canonical(z[1, i], z[3, i], z[5, i])
        p1 = canonical(b.z[1, i], b.z[3, i], z[5, i])
        for a, u in ((0, ux[i]), (1, uy[i])):
            want = kfac * u
            assert abs(float(p1[a] - p0[a]) - want) <= 1e-11 * abs(want) + 1e-19


def test_trwake_kick_linear_and_zero_slopes_exact(orc):
    rng = np.random.default_rng(6)
    n, nb = 500, 64
    z = rng.normal(0, 1e-3, (6, n))
    z[1] = 0.0
    z[3] = 0.0
    rg = np.array([z[4].min(), z[4].max()])
    vx, vy = np.zeros(nb), np.zeros(nb)
    b = orc.Beam(z, np.arange(n, dtype=np.uint32), np.full(n, -1, np.int64))
    orc.trwake_kick(b, rg, vx, vy, 1e-3)
    assert not b.z[1].any() and not b.z[3].any()          # zero wake: exactly no kick
    vx, vy = rng.normal(0, 1, nb), rng.normal(0, 1, nb)
    out = []
    for k in (1e-7, 2e-7):
        b = orc.Beam(z, np.arange(n, dtype=np.uint32), np.full(n, -1, np.int64))
        orc.trwake_kick(b, rg, vx, vy, k)
        out.append(b.z[[1, 3]].copy())
    assert np.allclose(out[1], 2 * out[0], rtol=1e-9, atol=1e-22)


# ------------------------------------------------------------------ the element in tracking
def trwake_element(nb=128, A=1e16):
    return Element("TRWAKE", wake_A=A, wake_tau0=10e-12, wake_omega=2 * math.pi * 50e9,
                   charge=1e-9, nbins=nb)


def test_trwake_is_causal_in_tracking(orc):
    """Only the trailing half (s > 0) is displaced: every particle ahead of
    the last leading bin centre keeps x' = y' = 0 exactly, and the first
    trailing particles are deflected towards the displacement (sin > 0 at
    short lags for a positive amplitude)."""
    rng = np.random.default_rng(7)
    n, nb = 20000, 128
    z = np.zeros((6, n))
    z[4] = np.sort(np.concatenate([-rng.uniform(0, 1e-3, n // 2), rng.uniform(0, 1e-3, n // 2)]))
    z[5] = rng.normal(0, 1e-3, n)
    z[0, n // 2:] = 5e-4
    b = orc.Beam(z, np.arange(n, dtype=np.uint32), np.full(n, -1, np.int64))
    orc.track(b, [trwake_element(nb)], 1)
    width = z[4].max() - z[4].min()
    lead = z[4] < z[4].min() + (nb // 2 - 1.5) * width / nb
    assert lead.sum() > 0.45 * n
    order = np.argsort(b.id)
    xp = b.z[1][order]
    assert not xp[lead].any() and not b.z[3].any()
    # W(0) = 0: the first trailing bin feels nothing yet; beyond it, within
    # half a wake period, every particle is deflected towards +x
    first_trail = (z[4] > 3 * width / nb) & (z[4] < 0.3e-3)
    assert first_trail.sum() > 1000 and (xp[first_trail] > 0).all()


def test_trwake_in_tracking_is_the_composed_steps(orc):
    rng = np.random.default_rng(8)
    n, nb = 5000, 256
    d = inputs.gaussian_beam(n, seed=8)
    d["z"][0] += 2e-4
    e = trwake_element(nb)
    b = orc.Beam.from_inputs(d)
    P = 3e8
    orc.track(b, [e], 1, p_ref=P)
    z = d["z"].copy()
    rg, cnt, dx, dy = orc.dipole_histogram(z[4], z[0], z[2], d["lost_at"], nb)
    w = orc.trwake_table(rg[0], rg[1], nb, e.wake_tau0, e.wake_omega)
    vx = orc.convolve_f64(orc.dipole_metres(dx), w)
    vy = orc.convolve_f64(orc.dipole_metres(dy), w)
    m = orc.Beam.from_inputs(d)
    orc.trwake_kick(m, rg, vx, vy, ((e.charge / n) * e.wake_A) / P)
    assert np.array_equal(b.z, m.z)
    assert np.abs(b.z[1] - z[1]).max() > 1e-9               # the wake does act
