"""Pins of the oracle's element maps against closed forms, independent
numerical integration and exact geometry.

Coordinates are (x, x', y, y', s, delta).  Canonical coordinates used for the
symplecticity checks are (x, px, y, py, -s, delta), px = x'(1+delta)/sqrt(1+x'^2+y'^2).
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_1710_07350_amd.inputs import Element, chicane_coef

mp.mp.dps = 40


def run(orc, lattice, z, passes=1, p_ref=1e9, seed=0):
    z = np.array(z, dtype=np.float64).reshape(6, -1)
    n = z.shape[1]
    b = orc.Beam(z, np.arange(n, dtype=np.uint32), np.full(n, -1, np.int64))
    orc.track(b, lattice, passes, p_ref=p_ref, seed=seed)
    return b


def to_canon(z):
    x, xp, y, yp, s, d = z
    f = (1.0 + d) / np.sqrt(1.0 + xp * xp + yp * yp)
    return np.array([x, xp * f, y, yp * f, -s, d])


def from_canon(w):
    x, px, y, py, ms, d = w
    pz = np.sqrt((1.0 + d) ** 2 - px * px - py * py)
    return np.array([x, px / pz, y, py / pz, -ms, d])


J6 = np.zeros((6, 6))
for _i in range(3):
    J6[2 * _i, 2 * _i + 1] = 1.0
    J6[2 * _i + 1, 2 * _i] = -1.0


def canon_jacobian(orc, elem, w0, h=1e-7):
    cols = []
    for j in range(6):
        wp = np.array(w0, dtype=float)
        wm = np.array(w0, dtype=float)
        wp[j] += h
        wm[j] -= h
        zs = np.stack([from_canon(wp), from_canon(wm)], axis=1)
        b = run(orc, [elem], zs)
        cp = to_canon(b.z[:, 0])
        cm = to_canon(b.z[:, 1])
        cols.append((cp - cm) / (2 * h))
    return np.array(cols).T


# ------------------------------------------------------------------ drift
def test_exact_drift_matches_paper_formula(orc):
    rng = np.random.default_rng(1)
    z = rng.normal(0, [[1e-3], [2e-3], [1e-3], [2e-3], [1e-3], [1e-3]], (6, 200))
    L = 1.37
    b = run(orc, [Element("EDRIFT", L=L)], z)
    for i in range(200):
        xp, yp = mp.mpf(z[1, i]), mp.mpf(z[3, i])
        # paper: s += L sqrt(1 + x'^2 + y'^2); deviation = that minus L
        ds = L * mp.sqrt(1 + xp * xp + yp * yp) - L
        assert abs(float(mp.mpf(b.z[4, i]) - (mp.mpf(z[4, i]) + ds))) <= 2e-16 * max(abs(z[4, i]), 1e-3)
        assert b.z[0, i] == pytest.approx(z[0, i] + z[1, i] * L, rel=1e-15, abs=1e-19)
    assert np.array_equal(b.z[[1, 3, 5]], z[[1, 3, 5]])


def test_exact_drift_equals_canonical_drift(orc):
    # the KQUAD integrator at k1 = 0 is three canonical drifts of total length L
    rng = np.random.default_rng(2)
    z = rng.normal(0, [[1e-3], [1e-3], [1e-3], [1e-3], [1e-3], [1e-3]], (6, 100))
    a = run(orc, [Element("EDRIFT", L=0.8)], z)
    c = run(orc, [Element("KQUAD", L=0.8, k=0.0, nsteps=1)], z)
    assert np.allclose(a.z, c.z, rtol=0, atol=4e-18)


# ------------------------------------------------------------------ QUAD map
def quad_ode(L, k1, delta):
    """R(delta) and the path quadratic form by integrating x'' = -K x, y'' = K y
    with K = k1/(1+delta), s' = (x'^2 + y'^2)/2 (paraxial)."""
    K = k1 / (1.0 + delta)

    def f(t, u):
        M = u[:4].reshape(2, 2)      # x-plane matrix
        N = u[4:8].reshape(2, 2)     # y-plane matrix
        A = np.array([[0, 1], [-K, 0]])
        B = np.array([[0, 1], [K, 0]])
        dM = A @ M
        dN = B @ N
        qx = 0.5 * np.outer(M[1], M[1])
        qy = 0.5 * np.outer(N[1], N[1])
        return np.concatenate([dM.ravel(), dN.ravel(), qx.ravel(), qy.ravel()])

    u0 = np.concatenate([np.eye(2).ravel(), np.eye(2).ravel(), np.zeros(8)])
    sol = solve_ivp(f, (0, L), u0, method="DOP853", rtol=1e-13, atol=1e-16)
    u = sol.y[:, -1]
    return u[:4].reshape(2, 2), u[4:8].reshape(2, 2), u[8:12].reshape(2, 2), u[12:16].reshape(2, 2)


def pair(j, k):
    idx = 0
    for a in range(6):
        for b in range(a, 6):
            if (a, b) == (j, k):
                return idx
            idx += 1


@pytest.mark.parametrize("k1", [1.2, -1.2, 0.35])
def test_quad_coefficients_vs_ode(orc, k1):
    L = 0.2 if abs(k1) > 1 else 0.7
    c = orc.quad_coef(L, k1)
    R = c[6:42].reshape(6, 6)
    T = c[42:].reshape(6, 21)
    Mx, My, Qx, Qy = quad_ode(L, k1, 0.0)
    h = 1e-4
    Mxp, Myp, _, _ = quad_ode(L, k1, h)
    Mxm, Mym, _, _ = quad_ode(L, k1, -h)
    dMx, dMy = (Mxp - Mxm) / (2 * h), (Myp - Mym) / (2 * h)
    assert np.allclose(R[0:2, 0:2], Mx, rtol=0, atol=1e-12)
    assert np.allclose(R[2:4, 2:4], My, rtol=0, atol=1e-12)
    for i in range(2):
        for j in range(2):
            assert T[i, pair(j, 5)] == pytest.approx(dMx[i, j], abs=1e-7)
            assert T[2 + i, pair(2 + j, 5)] == pytest.approx(dMy[i, j], abs=1e-7)
    assert T[4, pair(0, 0)] == pytest.approx(Qx[0, 0], abs=1e-12)
    assert T[4, pair(0, 1)] == pytest.approx(2 * Qx[0, 1], abs=1e-12)
    assert T[4, pair(1, 1)] == pytest.approx(Qx[1, 1], abs=1e-12)
    assert T[4, pair(2, 2)] == pytest.approx(Qy[0, 0], abs=1e-12)
    assert T[4, pair(2, 3)] == pytest.approx(2 * Qy[0, 1], abs=1e-12)
    assert T[4, pair(3, 3)] == pytest.approx(Qy[1, 1], abs=1e-12)
    # nothing else
    assert np.count_nonzero(c[:6]) == 0
    assert np.count_nonzero(R) == 10 and np.count_nonzero(T) == 14


@pytest.mark.parametrize("coef", ["quad", "chicane"])
def test_first_order_map_symplectic(orc, coef):
    c = orc.quad_coef(0.2, 1.2) if coef == "quad" else chicane_coef()
    R = c[6:42].reshape(6, 6)
    assert np.allclose(R.T @ J6 @ R, J6, atol=1e-14)


def test_chicane_closed_form(orc):
    rng = np.random.default_rng(3)
    z = rng.normal(0, 1e-2, (6, 50))
    b = run(orc, [Element("MAP2", coef=chicane_coef(-0.05, 0.075))], z)
    s_exact = z[4] + (-0.05) * z[5] + 0.075 * z[5] ** 2
    assert np.allclose(b.z[4], s_exact, rtol=1e-15, atol=1e-19)
    for k in (0, 1, 2, 3, 5):
        assert np.array_equal(b.z[k], z[k])


def test_linear_map_transports_second_moments(orc):
    """Sigma' = R Sigma R^T and mean' = R mean for any linear map."""
    rng = np.random.default_rng(4)
    z = rng.normal(0, 1e-3, (6, 5000)) + rng.normal(0, 1e-4, (6, 1))
    R = np.eye(6) + rng.normal(0, 0.3, (6, 6))
    c = np.zeros(168)
    c[6:42] = R.ravel()
    b0 = orc.Beam(z, np.arange(5000, dtype=np.uint32), np.full(5000, -1, np.int64))
    m0 = orc.moments(b0)
    b1 = run(orc, [Element("MAP2", coef=c)], z)
    m1 = orc.moments(b1)
    S0 = np.zeros((6, 6))
    S1 = np.zeros((6, 6))
    o = 7
    for k in range(6):
        for l in range(k, 6):
            S0[k, l] = S0[l, k] = m0[o]
            S1[k, l] = S1[l, k] = m1[o]
            o += 1
    assert np.allclose(m1[1:7], R @ m0[1:7], rtol=1e-12, atol=1e-18)
    ref = R @ S0 @ R.T
    assert np.allclose(S1, ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


# ------------------------------------------------------------------ thin multipole
def test_thin_sextupole_closed_form(orc):
    rng = np.random.default_rng(6)
    z = rng.normal(0, [[2e-3], [1e-4], [2e-3], [1e-4], [1e-3], [1e-3]], (6, 100))
    k2l = 5.0
    b = run(orc, [Element("MULT", k=k2l, order=2)], z)
    for i in range(100):
        x, xp, y, yp, d = (mp.mpf(z[k, i]) for k in (0, 1, 2, 3, 5))
        pz0 = (1 + d) / mp.sqrt(1 + xp * xp + yp * yp)
        px = xp * pz0 - k2l / 2 * (x * x - y * y)
        py = yp * pz0 + k2l * x * y
        pz = mp.sqrt((1 + d) ** 2 - px * px - py * py)
        # rounding scales with the terms added (x' and the kick), not the sum
        sx = abs(float(xp)) + abs(float(k2l / 2 * (x * x - y * y)))
        sy = abs(float(yp)) + abs(float(k2l * x * y))
        assert abs(float(px / pz - b.z[1, i])) <= 4e-16 * sx
        assert abs(float(py / pz - b.z[3, i])) <= 4e-16 * sy
    for k in (0, 2, 4, 5):
        assert np.array_equal(b.z[k], z[k])


def test_thin_multipole_orders(orc):
    # order 1 is a thin quadrupole: Delta px = -k1L x, Delta py = +k1L y
    z = np.array([[1e-3], [0.0], [2e-3], [0.0], [0.0], [0.0]])
    b = run(orc, [Element("MULT", k=0.5, order=1)], z)
    px, py = -0.5e-3, 1.0e-3
    pz = math.sqrt(1.0 - px * px - py * py)
    assert b.z[1, 0] == pytest.approx(px / pz, rel=1e-14)
    assert b.z[3, 0] == pytest.approx(py / pz, rel=1e-14)
    # order 3 (octupole): Delta px - i Delta py = -(k3L/6)(x+iy)^3
    z = np.array([[1e-2], [0.0], [5e-3], [0.0], [0.0], [0.0]])
    b = run(orc, [Element("MULT", k=60.0, order=3)], z)
    w = -(60.0 / 6.0) * (1e-2 + 5e-3j) ** 3
    pz = math.sqrt(1.0 - w.real ** 2 - w.imag ** 2)
    assert b.z[1, 0] == pytest.approx(w.real / pz, rel=1e-13)
    assert b.z[3, 0] == pytest.approx(-w.imag / pz, rel=1e-13)


@pytest.mark.parametrize("elem", [
    Element("MULT", k=5.0, order=2),
    Element("KQUAD", L=0.3, k=0.8, nsteps=1),
    Element("KQUAD", L=0.3, k=-0.8, nsteps=2),
    Element("CSBEND", L=1.5, angle=2 * math.pi / 80, nsteps=1),
    Element("EDRIFT", L=0.5),
])
def test_symplectic_in_canonical_variables(orc, elem):
    w0 = np.array([2e-3, 1e-3, -1e-3, 5e-4, 1e-3, 2e-3])
    M = canon_jacobian(orc, elem, w0)
    assert np.abs(M.T @ J6 @ M - J6).max() < 2e-7


# ------------------------------------------------------------------ kick-drift quad
def test_kquad_linear_limit_matches_thick_quad(orc):
    # small amplitudes, delta = 0, many steps: the linear cos/sin matrix
    L, k1 = 0.3, 0.8
    z = np.array([[1e-7], [2e-8], [-1e-7], [1e-8], [0.0], [0.0]])
    b = run(orc, [Element("KQUAD", L=L, k=k1, nsteps=16)], z)
    w = math.sqrt(k1)
    cx, sx = math.cos(w * L), math.sin(w * L)
    ch, sh = math.cosh(w * L), math.sinh(w * L)
    x = cx * 1e-7 + sx / w * 2e-8
    xp = -w * sx * 1e-7 + cx * 2e-8
    y = ch * -1e-7 + sh / w * 1e-8
    yp = w * sh * -1e-7 + ch * 1e-8
    assert b.z[0, 0] == pytest.approx(x, rel=1e-9)
    assert b.z[1, 0] == pytest.approx(xp, rel=1e-9)
    assert b.z[2, 0] == pytest.approx(y, rel=1e-9)
    assert b.z[3, 0] == pytest.approx(yp, rel=1e-9)


@pytest.mark.parametrize("kind", ["KQUAD", "CSBEND"])
def test_fourth_order_convergence(orc, kind):
    z = np.array([[3e-3], [2e-3], [-2e-3], [1e-3], [0.0], [5e-3]])
    if kind == "KQUAD":
        mk = lambda n: Element("KQUAD", L=1.0, k=3.0, nsteps=n)
    else:
        mk = lambda n: Element("CSBEND", L=1.5, angle=0.6, nsteps=n)
    ref = run(orc, [mk(256)], z).z[:, 0]
    errs = [np.abs(run(orc, [mk(n)], z).z[:, 0] - ref).max() for n in (2, 4, 8)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12.0 < r1 < 20.0 and 12.0 < r2 < 20.0, (errs, r1, r2)


@pytest.mark.parametrize("kind", ["KQUAD", "CSBEND"])
def test_time_reversal(orc, kind):
    z = np.array([[2e-3], [1e-3], [-1e-3], [2e-4], [1e-3], [1e-3]])
    if kind == "KQUAD":
        fw, bw = Element("KQUAD", L=0.3, k=0.8), Element("KQUAD", L=-0.3, k=0.8)
    else:
        a = 2 * math.pi / 80
        fw, bw = Element("CSBEND", L=1.5, angle=a), Element("CSBEND", L=-1.5, angle=-a)
    b = run(orc, [fw, bw], z)
    assert np.allclose(b.z[:, 0], z[:, 0], rtol=0, atol=2e-16)


def circle_exit(x0, xp0, y0, yp0, s0, d, rho, theta):
    """Exact sector-bend exit coordinates from circle geometry (mpmath)."""
    x0, xp0, y0, yp0, d = (mp.mpf(v) for v in (x0, xp0, y0, yp0, d))
    rho, theta = mp.mpf(rho), mp.mpf(theta)
    f = (1 + d) / mp.sqrt(1 + xp0 ** 2 + yp0 ** 2)
    px, py = xp0 * f, yp0 * f
    ph = mp.sqrt((1 + d) ** 2 - py ** 2)
    pzh = mp.sqrt(ph ** 2 - px ** 2)
    vx, vz = px / ph, pzh / ph
    r = rho * ph
    # coordinates (X radial outward, Z along the beam), bend centre at (-rho, 0)
    cx, cz = x0 - r * vz, r * vx
    psi0 = mp.atan2(-vx, vz)

    def cross(psi):
        X = cx + r * mp.cos(psi0 + psi) + rho
        Z = cz + r * mp.sin(psi0 + psi)
        return X * mp.sin(theta) - Z * mp.cos(theta)

    psi = mp.findroot(cross, theta)
    X = cx + r * mp.cos(psi0 + psi) + rho
    Z = cz + r * mp.sin(psi0 + psi)
    xe = X * mp.cos(theta) + Z * mp.sin(theta) - rho
    tx, tz = -mp.sin(psi0 + psi), mp.cos(psi0 + psi)
    pxe = ph * (tx * mp.cos(theta) + tz * mp.sin(theta))
    pze = ph * (-tx * mp.sin(theta) + tz * mp.cos(theta))
    l3 = r * psi * (1 + d) / ph
    return [xe, pxe / pze, y0 + rho * psi * py, py / pze, s0 + l3 - rho * theta, d]


def test_csbend_converges_to_circle(orc):
    L, ang = 1.5, 2 * math.pi / 80
    rho = L / ang
    z0 = [1e-3, 1e-3, 5e-4, -2e-4, 0.0, 1e-3]
    exact = np.array([float(v) for v in circle_exit(*z0, rho, ang)])
    errs = []
    for n in (1, 2, 4, 8):
        b = run(orc, [Element("CSBEND", L=L, angle=ang, nsteps=n)], np.array(z0).reshape(6, 1))
        errs.append(np.abs(b.z[:, 0] - exact).max())
    assert errs[-1] < 1e-9
    for a, b_ in zip(errs, errs[1:]):
        assert 14.0 < a / b_ < 18.0, errs          # fourth order: x16 per halving
    # the reference particle returns to the axis within the integrator error
    ref = [np.abs(run(orc, [Element("CSBEND", L=L, angle=ang, nsteps=n)],
                      np.zeros((6, 1))).z[:, 0]).max() for n in (4, 8)]
    assert ref[1] < 1e-9 and 14.0 < ref[0] / ref[1] < 18.0, ref


# ------------------------------------------------------------------ RF
def test_rf_cavity(orc):
    V, ph, f, P = 20e6, math.radians(-20.0), 1.3e9, 100e6
    rng = np.random.default_rng(8)
    z = np.zeros((6, 101))
    z[4, 1:] = rng.normal(0, 1e-3, 100)
    z[5, 1:] = rng.normal(0, 1e-3, 100)
    b = run(orc, [Element("RFCA", volt=V, phase=ph, freq=f)], z, p_ref=P)
    assert b.z[5, 0] == 0.0                     # reference particle keeps delta = 0 exactly
    k = 2 * mp.pi * f / 299792458
    Pn = P + V * mp.cos(ph)
    for i in range(1, 101):
        s, d = mp.mpf(z[4, i]), mp.mpf(z[5, i])
        exact = (P * (1 + d) + V * mp.cos(ph + k * s)) / Pn - 1
        assert abs(float(exact - b.z[5, i])) < 1e-15 * max(abs(float(exact)), 1e-3)
    # linear chirp at s -> 0: d delta/ds = -(V/P') k sin(phi)
    zz = np.zeros((6, 2))
    zz[4] = [1e-9, -1e-9]
    b = run(orc, [Element("RFCA", volt=V, phase=ph, freq=f)], zz, p_ref=P)
    slope = (b.z[5, 0] - b.z[5, 1]) / 2e-9
    assert slope == pytest.approx(float(-(V / Pn) * k * mp.sin(ph)), rel=1e-6)


def test_rf_reference_momentum_sequence(orc):
    # two cavities: the second sees P + V cos(phi) as its reference
    V, ph, f, P = 20e6, math.radians(-20.0), 1.3e9, 100e6
    cav = Element("RFCA", volt=V, phase=ph, freq=f)
    z = np.array([[0.0], [0.0], [0.0], [0.0], [1e-3], [0.0]])
    b = run(orc, [cav, cav], z, p_ref=P)
    k = 2 * mp.pi * f / 299792458
    P1 = P + V * mp.cos(ph)
    P2 = P1 + V * mp.cos(ph)
    d1 = (P + V * mp.cos(ph + k * mp.mpf(1e-3))) / P1 - 1
    d2 = (P1 * (1 + d1) + V * mp.cos(ph + k * mp.mpf(1e-3))) / P2 - 1
    assert b.z[5, 0] == pytest.approx(float(d2), rel=1e-13)


# ------------------------------------------------------------------ apertures
def test_apertures_brute_force(orc):
    X, Y = 5e-3, 4e-3
    pts = np.array([[0, 0], [X, 0], [-X, 0], [0, Y], [np.nextafter(X, 0), 0],
                    [X * 0.999, Y * 0.999], [np.nan, 0], [0, np.inf], [6e-3, 0]]).T
    z = np.zeros((6, pts.shape[1]))
    z[0], z[2] = pts
    b = run(orc, [Element("MARKER", aperture="RECT", ax=X, ay=Y)], z)
    alive_ids = set(b.id[b.lost_at < 0].tolist())
    assert alive_ids == {0, 4, 5}
    a, bb = 10e-3, 5e-3
    pts = np.array([[0, 0], [a, 0], [0, bb], [a * 0.7, bb * 0.7], [a * 0.7, bb * 0.72],
                    [np.nan, 0]]).T
    z = np.zeros((6, pts.shape[1]))
    z[0], z[2] = pts
    b = run(orc, [Element("MARKER", aperture="ELLIPSE", ax=a, ay=bb)], z)
    assert set(b.id[b.lost_at < 0].tolist()) == {0, 3}
