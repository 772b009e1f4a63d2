"""Analytic bispectrum of the paper's model field and its multipoles.

Test infrastructure only: nothing outside ``tests/``, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py`` may import this package.

* Eq. 15: real-space bispectrum of delta_G + f (delta_G^2 - <delta_G^2>) to
  first order in f:  B_r = 2 f [P1 P2 + P2 P3 + P3 P1].
* Eq. 17: linear RSD along z multiplies it by prod_i (1 + beta mu_i^2).
* Eq. 4: continuum multipoles [B_l^m]_c by quadrature over the orientation
  p (Gauss-Legendre in cos(theta) x uniform phi; the angular factor of Eq. 17
  is a polynomial of degree 6 in p, times Y of degree <= l, so a rule exact
  to degree 6 + l integrates it exactly), with mu_i from Eq. 3.
* Discrete prediction [B_l^m]_d (Sec. III.C): Eq. 17 at each combination's
  mean-value sides (mu_i = n_i / k_i), binned with Eq. 13 exactly like the
  estimator (same N_tri and Y weights).

The closed forms of the paper's Eq. 4 reference are not reproduced; the
quadrature replaces them.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import Geometry
from .ylm import norm_lm, assoc_legendre


def power(k, amp: float, n_s: float):
    """P(k) = A k^n_s (k in units of k_f), zero at k = 0."""
    k = np.asarray(k, dtype=np.float64)
    with np.errstate(divide="ignore"):
        out = amp * np.where(k > 0, k, 1.0) ** n_s
    return np.where(k > 0, out, 0.0)


def bispectrum_real(k1, k2, k3, amp: float, n_s: float, f_ng: float):
    """Eq. 15."""
    p1, p2, p3 = power(k1, amp, n_s), power(k2, amp, n_s), power(k3, amp, n_s)
    return 2.0 * f_ng * (p1 * p2 + p2 * p3 + p3 * p1)


def kaiser_factor(mu1, mu2, mu3, beta: float):
    """Angular factor of Eq. 17."""
    return (1.0 + beta * mu1 ** 2) * (1.0 + beta * mu2 ** 2) * (1.0 + beta * mu3 ** 2)


def orientation_cosines(pz, px, mu: float, t: float):
    """mu_1, mu_2, mu_3 of Eq. 3 for orientation p and shape (mu, t)."""
    s = math.sqrt(max(0.0, 1.0 - mu * mu))
    mu1 = pz
    mu2 = -mu * pz + s * px
    mu3 = -((1.0 - t * mu) * pz + t * s * px) / math.sqrt(1.0 - 2.0 * t * mu + t * t)
    return mu1, mu2, mu3


def continuum_multipole(l: int, m: int, mu: float, t: float, beta: float, n_theta: int = 24, n_phi: int = 48):
    """[B_l^m]_c / B_r(k1, mu, t): Eq. 4 with Eq. 17's angular factor.

    Returned in units of the real-space bispectrum, so it depends on shape
    only.  Complex in general; real for this model (mirror symmetry in p_y).
    """
    x, wx = np.polynomial.legendre.leggauss(n_theta)
    phi = 2.0 * np.pi * np.arange(n_phi) / n_phi
    ct = x[:, None]
    st = np.sqrt(1.0 - ct * ct)
    pz = ct * np.ones_like(phi)[None, :]
    px = st * np.cos(phi)[None, :]
    mu1, mu2, mu3 = orientation_cosines(pz, px, mu, t)
    ang = kaiser_factor(mu1, mu2, mu3, beta)
    ystar = norm_lm(l, abs(m)) * assoc_legendre(l, abs(m), pz) * np.exp(-1j * abs(m) * phi)[None, :]
    if m < 0:
        ystar = ((-1) ** abs(m)) * np.conj(ystar)
    integral = np.sum(wx[:, None] * ystar * ang) * (2.0 * np.pi / n_phi)
    return math.sqrt((2 * l + 1) / (4.0 * math.pi)) * integral


def side_cosines(geom: Geometry):
    """k_i and mu_i = n_i / k_i of each kept combination's three sides."""
    s = geom.combos.sides
    ksq = geom.sides.ksq[s]
    k = np.sqrt(ksq)
    n = geom.sides.plane[s].astype(np.float64)
    return k, n / k


def discrete_prediction(geom: Geometry, amp: float, n_s: float, f_ng: float, beta: float):
    """[B_l^m]_d per bin: Eq. 17 at combination means, binned with Eq. 13.

    Returns an array (n_lm, n_k1, n_mu, n_t), NaN where the bin is empty.
    """
    b = geom.binning
    c = geom.combos
    k, mus = side_cosines(geom)
    bs = bispectrum_real(k[:, 0], k[:, 1], k[:, 2], amp, n_s, f_ng) * kaiser_factor(
        mus[:, 0], mus[:, 1], mus[:, 2], beta
    )
    lms = b.lms()
    nb = b.n_bins
    nt = c.ntri.astype(np.float64)
    out = np.full((len(lms), nb), np.nan)
    for j, (l, m) in enumerate(lms):
        num = np.zeros(nb)
        den = np.zeros(nb)
        np.add.at(num, c.bin, c.w[:, j] * bs * nt)
        np.add.at(den, c.bin, c.d[:, j] * nt)
        ok = den > 0
        # odd l report the imaginary part of Eq. 13 (the estimator's reading);
        # the model bispectrum is real, so that part is zero
        part = np.zeros(nb) if l % 2 else num
        out[j, ok] = math.sqrt((2 * l + 1) / (4.0 * math.pi)) * part[ok] / den[ok]
    return out.reshape(len(lms), b.n_k1, b.n_mu, b.n_t)
