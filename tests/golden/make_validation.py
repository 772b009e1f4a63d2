"""Write the analytic predictions for the paper's validation setup.

Calls only the oracle (float64, CPU):  python tests/golden/make_validation.py
Setup (Sec. III.B-D of the paper): L = 215 Mpc, N_g = 384, P(k) ~ k^-2 with
sigma_G = 0.4 (f_NG sigma_G ~ 0.2), f_NG = 0.5, beta_1 = 1; one k1 bin
k1 = 2.1 +- 0.1 Mpc^-1; (mu, t) bins 12 x 12 (used for l <= 2), 8 x 8 (l = 4)
and 6 x 6 (l = 6).  Writes tests/golden/validation_ng384.npz with, per
binning, the triangle counts and two predictions (n_lm, 1, n, n):

* Bd: the paper's [B]_d, Eq. 17 at every combination's mean sides, binned
  with Eq. 13's weights;
* Bexact: the exact expectation of the estimator to first order in f_NG,
  i.e. Eq. 13 with every triangle's own B_s(q1, q2, q3) (Eqs. 15 and 17 at
  the triangle's integer modes) in place of the mean-side value.  The
  estimator is trilinear in the field, so this is the oracle estimator run
  on deterministic fields: with Delta_a = s_a P K and Delta_b = s_b K
  (P(m) = A |m|^n_s, K(m) = 1 + beta m_z^2 / |m|^2, s_a^2 s_b = 2 f_NG V),
  T(a + b) - T(a - b) = 6 T_sym(a, a, b) + 2 T(b), and 3 T_sym(a, a, b) sums
  Delta_a Delta_a Delta_b over the three slot assignments, which is
  V B_s per triangle.  s_a and s_b are balanced (s_a P ~ s_b at k1) so that
  no term is lost to cancellation.
"""
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.analytic import discrete_prediction  # noqa: E402
from oracle.estimator import estimate_streaming_binnings  # noqa: E402
from oracle.geometry import Binning, make_geometry  # noqa: E402
from synth import FieldRecipe, power_amplitude  # noqa: E402

NG, L = 384, 215.0
KF = 2.0 * math.pi / L
K1_MIN, K1_MAX = 2.0 / KF, 2.2 / KF
RECIPE = FieldRecipe(NG, box_len=L, n_s=-2.0, f_ng=0.5, beta=1.0, seed=0)
GRIDS = (12, 8, 6)


def binning(n):
    return Binning(NG, 1, K1_MIN, K1_MAX, n, n, box_len=L)


def main():
    amp = power_amplitude(RECIPE)
    out = {"k1": np.array([K1_MIN, K1_MAX]), "amp": np.array(amp)}
    for n in GRIDS:
        t0 = time.time()
        g = make_geometry(binning(n))
        bd = discrete_prediction(g, amp, RECIPE.n_s, RECIPE.f_ng, RECIPE.beta)
        out[f"Bd_{n}"] = bd
        out[f"counts_{n}"] = g.bin_counts().reshape(1, n, n)
        print(f"{n}x{n}: {len(g.combos.ntri)} combinations, {time.time() - t0:.0f} s", flush=True)
    for n, bex in zip(GRIDS, first_order_expectation(amp)):
        out[f"Bexact_{n}"] = bex
    np.savez_compressed(os.path.join(HERE, "validation_ng384.npz"), **out)


def deterministic_fields(amp):
    """Real fields whose Fourier modes (the oracle's Delta convention, V/N^3
    times the DFT) are s_a P K and s_b K."""
    m = np.fft.fftfreq(NG, d=1.0 / NG).round()
    m2 = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
    zero = m2 == 0
    m2s = np.where(zero, 1.0, m2)
    P = np.where(zero, 0.0, amp * m2s ** (RECIPE.n_s / 2.0))
    K = np.where(zero, 0.0, 1.0 + RECIPE.beta * m[None, None, :] ** 2 / m2s)
    del m2, m2s, zero
    vol = L ** 3
    c = (2.0 * RECIPE.f_ng * vol) ** (1.0 / 3.0)
    lam = (amp * (0.5 * (K1_MIN + K1_MAX)) ** RECIPE.n_s) ** (-1.0 / 3.0)
    Da = (c * lam) * P * K
    Db = (c / lam ** 2) * K
    del P, K

    def real_field(D):
        x = np.fft.ifftn(D) * (NG ** 3 / vol)
        return np.ascontiguousarray(x.real)

    return real_field(Da + Db), real_field(Da - Db), real_field(Db)


def first_order_expectation(amp):
    workers = int(os.environ.get("ORACLE_WORKERS", "8"))
    runs = []
    for name, field in zip(("a+b", "a-b", "b"), deterministic_fields(amp)):
        t0 = time.time()
        runs.append(estimate_streaming_binnings(field, [binning(n) for n in GRIDS], workers=workers, chunks=256))
        print(f"Bexact: field {name} in {time.time() - t0:.0f} s", flush=True)
    return [0.5 * (p.B - q.B) - r.B for p, q, r in zip(*runs)]


if __name__ == "__main__":
    main()
