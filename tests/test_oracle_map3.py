"""Pins of the oracle's third-order maps (the M3 matrix tracking of the
element table): the thick-quadrupole cubic coefficients against numerical
integration of the paraxial model, the evaluator against exact rational
arithmetic, the monomial index convention, and the order of accuracy."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_1710_07350_amd.inputs import Element
from test_oracle_elements import pair, quad_ode, run


def triple(j, k, l):
    idx = 0
    for a in range(6):
        for b in range(a, 6):
            for c in range(b, 6):
                if (a, b, c) == (j, k, l):
                    return idx
                idx += 1


TRIPLES = [(a, b, c) for a in range(6) for b in range(a, 6) for c in range(b, 6)]
PAIRS = [(a, b) for a in range(6) for b in range(a, 6)]


@pytest.mark.parametrize("k1", [1.2, -1.2, 0.8, -0.3])
def test_quad3_cubic_coefficients_vs_ode(orc, k1):
    """U_ij66 = R_ij''(delta)/2 and U_5jk6 = T_5jk'(delta) by differences of
    the integrated paraxial model, Richardson-extrapolated."""
    L = 0.2 if abs(k1) > 1 else 0.7
    c = orc.quad3_coef(L, k1)
    c2 = orc.quad_coef(L, k1)
    assert np.array_equal(c[:168], c2)
    U = c[168:].reshape(6, 56)

    def second(h):
        Mp, Np_, _, _ = quad_ode(L, k1, h)
        M0, N0, _, _ = quad_ode(L, k1, 0.0)
        Mm, Nm, _, _ = quad_ode(L, k1, -h)
        return (Mp - 2 * M0 + Mm) / (2 * h * h), (Np_ - 2 * N0 + Nm) / (2 * h * h)

    def first(h):
        _, _, Qxp, Qyp = quad_ode(L, k1, h)
        _, _, Qxm, Qym = quad_ode(L, k1, -h)
        return (Qxp - Qxm) / (2 * h), (Qyp - Qym) / (2 * h)

    h = 1e-2
    (ax, ay), (bx, by) = second(h), second(h / 2)
    Ux, Uy = (4 * bx - ax) / 3, (4 * by - ay) / 3
    (px, py), (qx, qy) = first(h), first(h / 2)
    dQx, dQy = (4 * qx - px) / 3, (4 * qy - py) / 3
    for i in range(2):
        for j in range(2):
            assert U[i, triple(j, 5, 5)] == pytest.approx(Ux[i, j], abs=1e-7)
            assert U[2 + i, triple(2 + j, 5, 5)] == pytest.approx(Uy[i, j], abs=1e-7)
    assert U[4, triple(0, 0, 5)] == pytest.approx(dQx[0, 0], abs=1e-7)
    assert U[4, triple(0, 1, 5)] == pytest.approx(2 * dQx[0, 1], abs=1e-7)
    assert U[4, triple(1, 1, 5)] == pytest.approx(dQx[1, 1], abs=1e-7)
    assert U[4, triple(2, 2, 5)] == pytest.approx(dQy[0, 0], abs=1e-7)
    assert U[4, triple(2, 3, 5)] == pytest.approx(2 * dQy[0, 1], abs=1e-7)
    assert U[4, triple(3, 3, 5)] == pytest.approx(dQy[1, 1], abs=1e-7)
    assert np.count_nonzero(U) == 14
    assert not orc.quad3_coef(L, 0.0)[168:].any()        # a drift has no chromatic terms


def test_map3_evaluator_exact_rational(orc):
    rng = np.random.default_rng(3)
    coef = rng.normal(0, 1, 504)
    coef[rng.random(504) < 0.3] = 0.0
    z = rng.normal(0, 1e-2, (6, 40))
    b = run(orc, [Element("MAP3", coef=coef)], z)
    C, R = coef[:6], coef[6:42].reshape(6, 6)
    T, U = coef[42:168].reshape(6, 21), coef[168:].reshape(6, 56)
    for p in range(z.shape[1]):
        q = [Fraction(float(v)) for v in z[:, p]]
        for i in range(6):
            terms = [Fraction(float(C[i]))]
            terms += [Fraction(float(R[i, j])) * q[j] for j in range(6)]
            terms += [Fraction(float(T[i, n])) * q[j] * q[k] for n, (j, k) in enumerate(PAIRS)]
            terms += [Fraction(float(U[i, n])) * q[j] * q[k] * q[l]
                      for n, (j, k, l) in enumerate(TRIPLES)]
            exact = sum(terms)
            bound = (len(terms) + 3) * 2.0 ** -53 * float(sum(abs(t) for t in terms))
            assert abs(float(Fraction(float(b.z[i, p])) - exact)) <= bound


def test_map3_monomial_convention(orc):
    """A map whose row 0 is the single cubic term z_j z_k z_l (other rows the
    identity) returns (z_j z_k) z_l exactly, for every triple."""
    rng = np.random.default_rng(4)
    z = rng.normal(0, 1, (6, 8))
    for n, (j, k, l) in enumerate(TRIPLES):
        coef = np.zeros(504)
        for i in range(1, 6):
            coef[6 + 7 * i] = 1.0
        coef[168 + n] = 1.0
        b = run(orc, [Element("MAP3", coef=coef)], z)
        assert np.array_equal(b.z[0], (z[j] * z[k]) * z[l]), (j, k, l)
        assert np.array_equal(b.z[1:], z[1:])


def paraxial_exact(L, k1, z0):
    """One particle through the paraxial quadrupole model with its own delta
    (no expansion in delta)."""
    x, xp, y, yp, s, d = z0
    K = k1 / (1.0 + d)

    def f(t, u):
        return [u[1], -K * u[0], u[3], K * u[2], 0.5 * (u[1] ** 2 + u[3] ** 2)]

    sol = solve_ivp(f, (0, L), [x, xp, y, yp, s], method="DOP853", rtol=2.5e-14, atol=1e-20)
    return np.append(sol.y[:, -1], d)


def test_quad3_is_third_order_accurate(orc):
    """Against the unexpanded model, the second-order map errs by O(delta^2)
    and the third-order map by O(delta^3): halving delta divides the errors
    by 4 and 8."""
    L, k1 = 0.2, 1.2
    errs = {2: [], 3: []}
    for d in (2e-2, 1e-2):
        z0 = np.array([[1e-3], [2e-4], [-8e-4], [1e-4], [0.0], [d]])
        ref = paraxial_exact(L, k1, z0[:, 0])
        for order in (2, 3):
            b = run(orc, [Element("QUAD", L=L, k=k1, order=order)], z0)
            errs[order].append(np.abs(b.z[:4, 0] - ref[:4]).max())
    r2 = errs[2][0] / errs[2][1]
    r3 = errs[3][0] / errs[3][1]
    assert 3.6 < r2 < 4.4, r2
    assert 7.0 < r3 < 9.0, r3
    assert errs[3][1] < 0.1 * errs[2][1]
