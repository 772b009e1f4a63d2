"""Spherical harmonics for the oracle, written from their textbook definition.

Test infrastructure only: nothing outside ``tests/``, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py`` may import this package.

Y_l^m(theta, phi) = N_lm P_l^m(cos theta) e^{i m phi}, with
N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and P_l^m carrying the
Condon-Shortley phase (-1)^m.  The paper defers the convention to its
Eq. 4 reference; the sign of B_2^1 it reports (Sec. III.D: positive for
mu < t, negative for mu > t) fixes the Condon-Shortley choice, which a test
pins through the analytic multipoles.

P_l is built from its explicit sum
    P_l(x) = 2^-l sum_k (-1)^k C(l,k) C(2l-2k, l) x^(l-2k)
and P_l^m(x) = (-1)^m (1-x^2)^(m/2) d^m/dx^m P_l(x), with the polynomial
coefficients kept as exact fractions until evaluation.  No recurrence is used,
so this code shares no arithmetic with any recurrence-based implementation.
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

import numpy as np


@lru_cache(maxsize=None)
def legendre_coeffs(l: int, m: int) -> tuple:
    """Exact coefficients c_j of d^m/dx^m P_l(x) = sum_j c_j x^j."""
    coeffs = [Fraction(0)] * (l + 1)
    for k in range(l // 2 + 1):
        c = Fraction((-1) ** k * math.comb(l, k) * math.comb(2 * l - 2 * k, l), 2 ** l)
        coeffs[l - 2 * k] += c
    for _ in range(m):
        coeffs = [coeffs[j] * j for j in range(1, len(coeffs))] or [Fraction(0)]
    return tuple(coeffs)


def assoc_legendre(l: int, m: int, x):
    """P_l^m(x) with the Condon-Shortley phase, for 0 <= m <= l (float64)."""
    if m < 0 or m > l:
        raise ValueError("need 0 <= m <= l")
    x = np.asarray(x, dtype=np.float64)
    poly = np.zeros_like(x)
    for c in reversed(legendre_coeffs(l, m)):
        poly = poly * x + float(c)
    sin_part = np.sqrt(np.maximum(0.0, 1.0 - x * x)) ** m
    return ((-1.0) ** m) * sin_part * poly


def norm_lm(l: int, m: int) -> float:
    """N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!)."""
    return math.sqrt((2 * l + 1) / (4.0 * math.pi) * math.factorial(l - m) / math.factorial(l + m))


def ylm(l: int, m: int, theta, phi):
    """Complex Y_l^m(theta, phi); negative m via Y_l^-m = (-1)^m conj(Y_l^m)."""
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    am = abs(m)
    val = norm_lm(l, am) * assoc_legendre(l, am, np.cos(theta)) * np.exp(1j * am * phi)
    if m < 0:
        val = ((-1) ** am) * np.conj(val)
    return val


def lm_list(l_max: int = 6, m_max: int = 6, even_only: bool = True):
    """Output order of the multipoles: l ascending, then m = 0..min(l, m_max)."""
    out = []
    for l in range(l_max + 1):
        if even_only and l % 2:
            continue
        for m in range(min(l, m_max) + 1):
            out.append((l, m))
    return out
