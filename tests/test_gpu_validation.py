"""The paper's validation experiment (Sec. III.B-D) on the GPU estimator.

50 realisations of the non-Gaussian redshift-space field (L = 215 Mpc,
N_g = 384, P ~ k^-2, f_NG = 0.5, beta_1 = 1), all 16 multipoles in the k1 bin
2.1 +- 0.1 Mpc^-1 with 12 x 12 (mu, t) bins for l <= 2, 8 x 8 for l = 4 and
6 x 6 for l = 6, compared with the discrete analytic prediction [B]_d
(tests/golden/validation_ng384.npz, written by make_validation.py from the
oracle).  Delta = |mean - [B]_d| / sigma, sigma the rms of the ensemble mean.
The paper finds Delta <= 3 in most bins, a few at 3-5 and rare 5-7 near the
squeezed corner, and monopole deviations within a few percent.  Fields come
from the torch port of the generator (same recipe, different random stream).
"""
import math
import os

import numpy as np
import pytest

from synth import FieldRecipe, make_field_torch

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
NG, L = 384, 215.0
N_REAL = 50
GRIDS = {12: (0, 2), 8: (4, 4), 6: (6, 6)}  # (mu, t) bins -> l range it serves


@pytest.mark.timeout(900)
def test_paper_validation_ensemble():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_14513_amd import bk

    gold = np.load(os.path.join(HERE, "golden", "validation_ng384.npz"))
    k1_min, k1_max = gold["k1"]
    stream = torch.cuda.current_stream().cuda_stream
    plans = {}
    try:
        for n in GRIDS:
            print(f"validation: plan {n}x{n}", flush=True)
            plans[n] = bk.Estimator(bk.make_binning(NG, 1, k1_min, k1_max, n, n, box_len=L), prec=bk.BK_F32)
            assert np.array_equal(plans[n].counts(), gold[f"counts_{n}"]), f"triangle counts differ ({n}x{n})"
        lms = plans[12].lm_list()
        samples = {n: [] for n in GRIDS}
        for s in range(N_REAL):
            f = make_field_torch(FieldRecipe(NG, box_len=L, n_s=-2.0, f_ng=0.5, beta=1.0, seed=1000 + s))
            f32 = f.to(torch.float32).contiguous()
            for n, est in plans.items():
                est.load(f32, stream)
                est.estimate(stream)
                samples[n].append(est.multipoles()[0])
            if s % 10 == 9:
                print(f"validation: {s + 1} realisations", flush=True)
    finally:
        for est in plans.values():
            est.close()

    lines, all_delta, mono_dev = [], [], []
    for n, (l_lo, l_hi) in GRIDS.items():
        X = np.stack(samples[n])  # (N_REAL, n_lm, 1, n, n)
        mean = X.mean(axis=0)
        sigma = X.std(axis=0, ddof=1) / math.sqrt(N_REAL)
        bd = gold[f"Bd_{n}"]
        for j, (l, m) in enumerate(lms):
            if not (l_lo <= l <= l_hi):
                continue
            ok = np.isfinite(bd[j]) & np.isfinite(mean[j]) & (sigma[j] > 0)
            d = np.abs(mean[j][ok] - bd[j][ok]) / sigma[j][ok]
            all_delta.append(d)
            if (l, m) == (0, 0):
                mono_dev = (mean[j][ok] / bd[j][ok] - 1.0)
            lines.append(f"l={l} m={m} ({n}x{n}): bins {d.size}, Delta<=3 {np.mean(d <= 3):.2f}, "
                         f"3-5 {np.mean((d > 3) & (d <= 5)):.2f}, max {d.max():.1f}")
    d = np.concatenate(all_delta)
    summary = (f"all multipoles: {d.size} bins, Delta<=3 {np.mean(d <= 3):.3f}, <=5 {np.mean(d <= 5):.3f}, "
               f"max {d.max():.1f}; B_0^0 fractional deviation median {np.median(np.abs(mono_dev)):.4f}, "
               f"range [{mono_dev.min():.4f}, {mono_dev.max():.4f}]")
    print("\n".join(lines + [summary]), flush=True)
    out = os.environ.get("BK_VALIDATION_REPORT")
    if out:
        with open(out, "w") as fh:
            fh.write("\n".join(lines + [summary]) + "\n")
    assert np.mean(d <= 3) >= 0.75, summary
    assert np.mean(d <= 5) >= 0.9, summary
    assert np.median(np.abs(mono_dev)) < 0.05, summary
