"""The continuum multipoles [B_l^m]_c of the model field (Eq. 4 with the
angular factor of Eq. 17), pinned by an exact symbolic evaluation that
shares nothing with the oracle's quadrature: sympy's own Y_l^m, the cosines
mu_i taken from the triangle's side vectors (Eq. 2: k1 along z, k2 in the x-z
plane at -k1.k2/(k1 k2) = mu with |k2| = t k1, k3 = -k1 - k2), the phi
integral from the binomial expansion of cos^k(phi), and the theta integral of
a polynomial in cos(theta) done exactly.  Both the oracle and the library's
host function must match it."""
import math

import numpy as np
import pytest

sp = pytest.importorskip("sympy")

from oracle.analytic import continuum_multipole  # noqa: E402

X, Z, U = sp.symbols("X Z U", real=True)
TH = sp.symbols("theta", real=True)


def _phi_integral(k, m):
    """Integral over [0, 2 pi) of cos^k(phi) exp(-i m phi)."""
    if k < m or (k - m) % 2:
        return sp.Integer(0)
    return 2 * sp.pi * sp.binomial(k, (k - m) // 2) / sp.Integer(2) ** k


def _exact(l, m, mu, t, beta):
    s = sp.sqrt(1 - mu ** 2)
    k1 = sp.Matrix([0, 0, 1])
    k2 = sp.Matrix([s, 0, -mu])  # unit vector; the side itself is t k1 long
    k3 = -(k1 + t * k2)
    k3 = k3 / sp.sqrt(k3.dot(k3))
    p = sp.Matrix([X, 0, Z])  # no side has a y component, so p_y drops out
    ang = sp.Poly(sp.expand(sp.prod([1 + beta * p.dot(k) ** 2 for k in (k1, k2, k3)])), X, Z)
    # Y_l^m(theta, phi) = Y_l^m(theta, 0) e^{i m phi}; p_x = sin(theta) cos(phi), p_z = cos(theta)
    y_theta = sp.Ynm(l, m, TH, 0).expand(func=True)
    y_u = y_theta.subs(sp.sin(TH), sp.sqrt(1 - U ** 2)).subs(sp.cos(TH), U)
    total = 0
    for (k, j), c in ang.terms():
        a = _phi_integral(k, m)
        if a != 0:
            total += c * a * sp.integrate(sp.expand(y_u * sp.sqrt(1 - U ** 2) ** k * U ** j), (U, -1, 1))
    return complex(sp.N(sp.sqrt(sp.Rational(2 * l + 1) / (4 * sp.pi)) * total, 30))


SHAPES = [(sp.Rational(3, 5), sp.Rational(4, 5)), (sp.Rational(1, 2), sp.Integer(1)),
          (sp.Rational(9, 10), sp.Rational(3, 5))]


@pytest.mark.parametrize("beta", [sp.Rational(1, 2), sp.Integer(1)])
@pytest.mark.parametrize("shape", range(len(SHAPES)))
def test_continuum_multipoles_equal_the_exact_integral(shape, beta):
    from paper_2405_14513_amd import bk

    mu, t = SHAPES[shape]
    host = bk.bk_continuum_multipoles(6, 6, float(mu), float(t), float(beta))
    lms = [(l, m) for l in range(0, 7, 2) for m in range(0, l + 1)]
    assert len(host) == len(lms)
    scale = abs(_exact(0, 0, mu, t, beta))
    for i, (l, m) in enumerate(lms):
        ref = _exact(l, m, mu, t, beta)
        assert abs(ref.imag) < 1e-25  # real for this model
        got = continuum_multipole(l, m, float(mu), float(t), float(beta))
        assert abs(got - ref.real) < 1e-13 * scale, (l, m, got, ref)
        assert abs(host[i] - ref.real) < 1e-13 * scale, (l, m, host[i], ref)


def test_odd_continuum_multipoles_vanish_exactly():
    """The angular factor is even in p, so every odd l integrates to zero."""
    mu, t = SHAPES[0]
    for l in (1, 3, 5):
        for m in range(0, l + 1):
            assert _exact(l, m, mu, t, sp.Integer(1)) == 0
            assert abs(continuum_multipole(l, m, float(mu), float(t), 1.0)) < 1e-14
