"""Write the discrete analytic prediction [B]_d for the paper's validation setup.

Calls only the oracle (float64, CPU):  python tests/golden/make_validation.py
Setup (Sec. III.B-D of the paper): L = 215 Mpc, N_g = 384, P(k) ~ k^-2 with
sigma_G = 0.4 (f_NG sigma_G ~ 0.2), f_NG = 0.5, beta_1 = 1; one k1 bin
k1 = 2.1 +- 0.1 Mpc^-1; (mu, t) bins 12 x 12 (used for l <= 2), 8 x 8 (l = 4)
and 6 x 6 (l = 6).  [B]_d is Eq. 17 at every combination's mean sides, binned
with Eq. 13's weights.  Writes tests/golden/validation_ng384.npz with, per
binning, [B]_d (n_lm, 1, n, n) and the triangle counts.
"""
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.analytic import discrete_prediction  # noqa: E402
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
    np.savez_compressed(os.path.join(HERE, "validation_ng384.npz"), **out)


if __name__ == "__main__":
    main()
