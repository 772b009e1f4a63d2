"""Seeded synthetic fields shaped like the paper's validation simulation.

This module only makes inputs.  It holds none of the estimator's arithmetic
and is shared by the oracle, the tests and the benchmark.

Recipe (Section III.A-B of the paper, Eqs. 14 and 16):

1. A Gaussian field g on an N_g^3 periodic grid with power spectrum
   P(k) = A |m|^n_s, where m is the integer wave vector (k = m k_f,
   k_f = 2 pi / L) and the zero mode is removed.  A is chosen so that the
   expected variance of g is sigma_G^2 (the paper runs f_NG sigma_G ~ 0.2
   with f_NG = 0.5, so sigma_G = 0.4).
2. Local quadratic non-Gaussianity: delta_r = g + f_NG (g^2 - <g^2>), with
   <g^2> the sample mean over the grid.
3. Linear (Kaiser) redshift-space distortion along z, the line of sight:
   Delta_s(m) = (1 + beta mu_m^2) Delta_r(m), mu_m = m_z / |m|, factor 0 at
   m = 0.

White noise comes from numpy's PCG64 ``default_rng(seed)``, one N(0,1) draw
per cell in C order, and all arithmetic is float64.  The Fourier convention
is numpy's (forward transform without normalisation).  With
Delta = (V / N_g^3) DFT(delta), the power spectrum of g is
P = <|Delta|^2> / V, which is what the amplitude below enforces.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class FieldRecipe:
    """Parameters of one synthetic realisation."""

    ng: int
    box_len: float | None = None  # L; defaults to N_g (cell = 1)
    n_s: float = -2.0  # power-law index of P(k)
    f_ng: float = 0.5  # quadratic coefficient (Eq. 14)
    beta: float = 0.5  # Kaiser parameter (Eq. 16)
    sigma_g: float = 0.4  # target rms of the Gaussian part
    seed: int = 0

    @property
    def length(self) -> float:
        return float(self.ng) if self.box_len is None else float(self.box_len)


def _int_freqs(ng: int) -> np.ndarray:
    """Signed integer wave numbers in numpy FFT order."""
    return np.fft.fftfreq(ng, d=1.0 / ng).round().astype(np.int64)


def power_amplitude(recipe: FieldRecipe) -> float:
    """A such that the expected variance of g equals sigma_g^2.

    Var(g) = (1/V) sum_{m != 0} P(m) = (A / V) sum_{m != 0} |m|^n_s, so
    A = sigma^2 V / sum_{m != 0} |m|^n_s (sum over the full DFT cube).
    """
    ng = recipe.ng
    f = _int_freqs(ng).astype(np.float64)
    m2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    m2[0, 0, 0] = 1.0
    mag = np.sqrt(m2) ** recipe.n_s
    mag[0, 0, 0] = 0.0
    vol = recipe.length ** 3
    return recipe.sigma_g ** 2 * vol / float(mag.sum())


def make_field(recipe: FieldRecipe) -> np.ndarray:
    """Return delta_s(x) as float64, shape (N_g, N_g, N_g), z (LoS) fastest."""
    ng = recipe.ng
    vol = recipe.length ** 3
    rng = np.random.default_rng(recipe.seed)
    white = rng.standard_normal((ng, ng, ng))

    f = _int_freqs(ng).astype(np.float64)
    fz = f[: ng // 2 + 1]
    m2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + fz[None, None, :] ** 2
    zero = m2 == 0.0
    m2s = np.where(zero, 1.0, m2)

    amp = power_amplitude(recipe)
    pk = amp * np.sqrt(m2s) ** recipe.n_s
    pk[zero] = 0.0
    # E|DFT(white)|^2 = N^3, so scaling by sqrt(P N^3 / V) gives <|Delta|^2>/V = P.
    g = np.fft.irfftn(np.fft.rfftn(white) * np.sqrt(pk * ng ** 3 / vol), s=(ng, ng, ng), axes=(0, 1, 2))

    delta_r = g + recipe.f_ng * (g * g - np.mean(g * g))

    kaiser = 1.0 + recipe.beta * (fz[None, None, :] ** 2) / m2s
    kaiser[zero] = 0.0
    delta_s = np.fft.irfftn(np.fft.rfftn(delta_r) * kaiser, s=(ng, ng, ng), axes=(0, 1, 2))
    return np.ascontiguousarray(delta_s)


def field_digest(delta: np.ndarray) -> str:
    """SHA-256 of the float64 bytes, used to check a regenerated field."""
    return hashlib.sha256(np.ascontiguousarray(delta, dtype=np.float64).tobytes()).hexdigest()


def plane_wave_field(ng: int, waves) -> np.ndarray:
    """Sum of real plane waves 2 A cos(2 pi m.x / N + phi).

    ``waves`` is a list of (m, A, phi) with m an integer 3-vector.  Used for
    closed-form checks: the DFT of one term is N^3 A e^{i phi} at m and its
    conjugate at -m.
    """
    idx = np.arange(ng, dtype=np.float64)
    x = idx[:, None, None]
    y = idx[None, :, None]
    z = idx[None, None, :]
    out = np.zeros((ng, ng, ng))
    for m, amp, phi in waves:
        arg = 2.0 * np.pi * (m[0] * x + m[1] * y + m[2] * z) / ng + phi
        out += 2.0 * amp * np.cos(arg)
    return out
