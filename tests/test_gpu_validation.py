"""The paper's validation experiment (Sec. III.B-D) on the GPU estimator.

50 realisations of the non-Gaussian redshift-space field (L = 215 Mpc,
N_g = 384, P ~ k^-2, beta_1 = 1), all 16 multipoles in the k1 bin
2.1 +- 0.1 Mpc^-1 with 12 x 12 (mu, t) bins for l <= 2, 8 x 8 for l = 4 and
6 x 6 for l = 6, from one plan with three resolutions, compared with the
discrete analytic prediction [B]_d of tests/golden/validation_ng384.npz
(written by make_validation.py from the oracle at f_NG = 0.5).
Delta = |mean - [B]_d| / sigma, sigma the rms of the ensemble mean.

Each Gaussian realisation g is used at f_NG = +-0.5 and +-0.25
(delta = g + f_NG (g^2 - <g^2>), Eq. 14).  The estimator is cubic in delta,
so for one realisation B_hat(f) = c0 + c1 f + c2 f^2 + c3 f^3, where c0 and
c2 (odd in g) have zero mean, c1 has the mean of Eq. 15's bispectrum and c3
that of the term third order in f_NG which Eq. 15 leaves out.  The odd part
(B_hat(f) - B_hat(-f)) / 2 = c1 f + c3 f^3 at two f_NG gives c1 and c3 per
realisation, free of the Gaussian noise c0.  Their ensemble means are
compared with Bexact (the exact first-order expectation of the estimator,
Eq. 13 over every triangle's own B_s, from the oracle) and with [B]_d.
Fields come from the torch port of the generator (same recipe, different
random stream).

With BK_VALIDATION_OUT set to a directory, the Delta_l^m (mu, t) maps, the
ensemble means, sigmas, [B]_d and Bexact, the first- and third-order
coefficients, and the three boundary curves of the (mu, t) plane (mu ~ 1,
t ~ 1, 2 mu t ~ 1) are written there as validation_ng384.npz, with a text
summary.
"""
import math
import os
import time

import numpy as np
import pytest

from synth import FieldRecipe, make_field_torch

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
NG, L = 384, 215.0
N_REAL = 50
F_NG = (0.5, -0.5, 0.25, -0.25)
F_GOLD = 0.5  # f_NG of the stored predictions (both are linear in f_NG)
GRIDS = ((12, (0, 2)), (8, (4, 4)), (6, (6, 6)))  # (mu, t) bins per axis, l range served; resolution order


def _boundaries(n, counts):
    """Bin indices (i_mu, i_t) along the mu ~ 1 edge (last mu bin, by t), the
    t ~ 1 edge (last t bin, by mu) and the 2 mu t ~ 1 edge (first non-empty t
    bin of every mu bin, by mu)."""
    mu1 = [(n - 1, it) for it in range(n) if counts[n - 1, it] > 0]
    t1 = [(im, n - 1) for im in range(n) if counts[im, n - 1] > 0]
    low = []
    for im in range(n):
        nz = np.nonzero(counts[im] > 0)[0]
        if nz.size:
            low.append((im, int(nz[0])))
    return {"mu1": mu1, "t1": t1, "2mut1": low}


@pytest.fixture(scope="module")
def ensemble():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_14513_amd import bk

    gold = np.load(os.path.join(HERE, "golden", "validation_ng384.npz"))
    k1_min, k1_max = gold["k1"]
    stream = torch.cuda.current_stream().cuda_stream
    print("validation: plan with 12x12, 8x8, 6x6 resolutions", flush=True)
    est = bk.Estimator(bk.make_binning(NG, 1, k1_min, k1_max, 12, 12, box_len=L), prec=bk.BK_F32,
                       extra_bins=[(1, 8, 8), (1, 6, 6)])
    samples = {f: [[] for _ in GRIDS] for f in F_NG}
    try:
        counts = [est.counts(r) for r in range(len(GRIDS))]
        means = [est.bin_means(r) for r in range(len(GRIDS))]
        lms = est.lm_list()
        t_est = 0.0
        for s in range(N_REAL):
            for f in F_NG:
                x = make_field_torch(FieldRecipe(NG, box_len=L, n_s=-2.0, f_ng=f, beta=1.0, seed=1000 + s))
                est.load(x.to(torch.float32).contiguous(), stream)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                est.estimate(stream)
                torch.cuda.synchronize()
                t_est += time.perf_counter() - t0
                for r in range(len(GRIDS)):
                    samples[f][r].append(est.multipoles(r)[0])
            if s % 10 == 9:
                print(f"validation: {s + 1} realisations x {len(F_NG)} f_NG", flush=True)
    finally:
        est.close()
    out = {"lms": lms, "counts": counts, "means": means, "gold": gold,
           "ms_per_estimate": 1e3 * t_est / (N_REAL * len(F_NG)), "stats": {}, "orders": {}}
    for r, (n, _) in enumerate(GRIDS):
        X = {f: np.stack(samples[f][r]) for f in F_NG}  # (N_REAL, n_lm, 1, n, n)
        bd1 = gold[f"Bd_{n}"] / F_GOLD  # per unit f_NG
        bx1 = gold[f"Bexact_{n}"] / F_GOLD
        for f in (0.5, 0.25):
            mean = X[f].mean(axis=0)
            sigma = X[f].std(axis=0, ddof=1) / math.sqrt(N_REAL)
            with np.errstate(invalid="ignore", divide="ignore"):
                delta = np.abs(mean - f * bd1) / sigma
                frac = mean / (f * bd1) - 1.0
            out["stats"][(f, n)] = {"mean": mean, "sigma": sigma, "bd": f * bd1, "bexact": f * bx1,
                                    "delta": delta, "frac": frac}
        o5 = 0.5 * (X[0.5] - X[-0.5])
        o25 = 0.5 * (X[0.25] - X[-0.25])
        c3 = (o5 / 0.5 - o25 / 0.25) / (0.5 ** 2 - 0.25 ** 2)
        c1 = o25 / 0.25 - 0.25 ** 2 * c3
        out["orders"][n] = {
            "c1": c1.mean(axis=0), "c1_sigma": c1.std(axis=0, ddof=1) / math.sqrt(N_REAL),
            "c3": c3.mean(axis=0), "c3_sigma": c3.std(axis=0, ddof=1) / math.sqrt(N_REAL),
            "bd1": bd1, "bexact1": bx1,
        }
    _write_outputs(out)
    return out


def _write_outputs(ens):
    target = os.environ.get("BK_VALIDATION_OUT")
    if not target:
        return
    os.makedirs(target, exist_ok=True)
    arrays = {"lms": np.array(ens["lms"]), "f_ng": np.array([0.5, 0.25]), "n_real": np.array(N_REAL)}
    for r, (n, _) in enumerate(GRIDS):
        c = ens["counts"][r][0]
        arrays[f"counts_{n}"] = c
        arrays[f"bin_means_{n}"] = ens["means"][r][0]
        bounds = _boundaries(n, c)
        for name, idx in bounds.items():
            arrays[f"boundary_{name}_{n}_bins"] = np.array(idx)
        for key, v in ens["orders"][n].items():
            arrays[f"{key}_{n}"] = v[:, 0]
        for f in (0.5, 0.25):
            st = ens["stats"][(f, n)]
            tag = f"{n}_f{f:g}"
            for key in ("mean", "sigma", "bd", "bexact", "delta"):
                arrays[f"{key}_{tag}"] = st[key][:, 0]
            for name, idx in bounds.items():
                ii = tuple(np.array(idx).T)
                for key in ("mean", "sigma", "bd", "bexact"):
                    arrays[f"boundary_{name}_{key}_{tag}"] = st[key][:, 0][(slice(None),) + ii]
    np.savez_compressed(os.path.join(target, "validation_ng384.npz"), **arrays)
    with open(os.path.join(target, "validation_ng384.txt"), "w") as fh:
        fh.write("\n".join(_summary_lines(ens)) + "\n")


def _orders_lines(ens):
    lines = []
    for n, (l_lo, l_hi) in GRIDS:
        o = ens["orders"][n]
        for j, (l, m) in enumerate(ens["lms"]):
            if not (l_lo <= l <= l_hi):
                continue
            ok = np.isfinite(o["bd1"][j]) & (o["c1_sigma"][j] > 0)
            z = (o["c1"][j][ok] - o["bexact1"][j][ok]) / o["c1_sigma"][j][ok]
            line = f"l={l} m={m} ({n}x{n}): first order vs Bexact |z| median {np.median(np.abs(z)):.2f} max {np.abs(z).max():.2f}"
            if l == 0:
                mv = o["bexact1"][j][ok] / o["bd1"][j][ok] - 1.0
                b1 = o["c1"][j][ok] / o["bexact1"][j][ok] - 1.0
                third = 0.25 * o["c3"][j][ok] / o["c1"][j][ok]
                line += (f"; c1/Bexact - 1 median {np.median(b1):+.4f}; Bexact/[B]_d - 1 median {np.median(mv):+.4f} "
                         f"range [{mv.min():+.4f}, {mv.max():+.4f}]; third-order share at f_NG=0.5 median "
                         f"{np.median(third):+.4f} range [{third.min():+.4f}, {third.max():+.4f}]")
            lines.append(line)
    return lines


def _summary_lines(ens):
    lines = [f"one estimate (three resolutions): {ens['ms_per_estimate']:.2f} ms"]
    for f in (0.5, 0.25):
        for n, (l_lo, l_hi) in GRIDS:
            st = ens["stats"][(f, n)]
            for j, (l, m) in enumerate(ens["lms"]):
                if not (l_lo <= l <= l_hi):
                    continue
                d = st["delta"][j]
                ok = np.isfinite(d)
                lines.append(f"f_NG={f:g} l={l} m={m} ({n}x{n}): bins {ok.sum()}, Delta<=3 {np.mean(d[ok] <= 3):.2f}, "
                             f"3-5 {np.mean((d[ok] > 3) & (d[ok] <= 5)):.2f}, >5 {np.sum(d[ok] > 5)}, "
                             f"max {d[ok].max():.1f}")
            fr = st["frac"][0, 0]
            ok = np.isfinite(fr)
            lines.append(f"f_NG={f:g} B_0^0 ({n}x{n}) fractional deviation from [B]_d: median |dev| "
                         f"{np.median(np.abs(fr[ok])):.4f}, range [{fr[ok].min():.4f}, {fr[ok].max():.4f}]")
    return lines + _orders_lines(ens) + _boundary_lines(ens)


def _boundary_lines(ens):
    """B_0^0 and B_2^0 along the three boundaries of the 12 x 12 (mu, t)
    plane at f_NG = 0.5: mean, sigma and [B]_d per bin (the right-hand
    panels of the paper's l = 0, 2 figure)."""
    lines = []
    st = ens["stats"][(0.5, 12)]
    c = ens["counts"][0][0]
    means = ens["means"][0][0]
    for name, idx in _boundaries(12, c).items():
        for l in (0, 2):
            j = ens["lms"].index((l, 0))
            cells = []
            for im, it in idx:
                cells.append(f"(mu {means[im, it, 1]:.3f}, t {means[im, it, 2]:.3f}) {st['mean'][j][0, im, it]:.4g} "
                             f"+- {st['sigma'][j][0, im, it]:.2g} vs {st['bd'][j][0, im, it]:.4g}")
            lines.append(f"boundary {name} l={l} m=0: " + "; ".join(cells))
    return lines


def _deltas(ens, f, l_filter=lambda l: True):
    out = []
    for n, (l_lo, l_hi) in GRIDS:
        st = ens["stats"][(f, n)]
        for j, (l, m) in enumerate(ens["lms"]):
            if l_lo <= l <= l_hi and l_filter(l):
                d = st["delta"][j]
                out.append(d[np.isfinite(d)])
    return np.concatenate(out)


def test_validation_counts_match_the_oracle(ensemble):
    for r, (n, _) in enumerate(GRIDS):
        assert np.array_equal(ensemble["counts"][r], ensemble["gold"][f"counts_{n}"]), f"triangle counts ({n}x{n})"


def test_validation_at_the_papers_f_ng(ensemble):
    """Sec. III.D at f_NG = 0.5: Delta <= 3 in most bins, a few at 3-5, rare
    ones up to 7."""
    print("\n".join(_summary_lines(ensemble)), flush=True)
    d = _deltas(ensemble, 0.5)
    assert np.mean(d <= 3) >= 0.90
    assert np.mean(d <= 5) >= 0.99
    assert d.max() <= 7.0
    d2 = _deltas(ensemble, 0.5, lambda l: l >= 2)
    assert np.mean(d2 <= 3) >= 0.95


def test_first_order_estimate_is_unbiased(ensemble):
    """The f_NG-linear part of the ensemble equals the estimator's exact
    first-order expectation in every multipole and bin, within its noise."""
    z_all = []
    for n, (l_lo, l_hi) in GRIDS:
        o = ensemble["orders"][n]
        for j, (l, m) in enumerate(ensemble["lms"]):
            if not (l_lo <= l <= l_hi):
                continue
            ok = np.isfinite(o["bd1"][j]) & (o["c1_sigma"][j] > 0)
            z_all.append((o["c1"][j][ok] - o["bexact1"][j][ok]) / o["c1_sigma"][j][ok])
    z = np.abs(np.concatenate(z_all))
    print(f"first order vs Bexact: {z.size} bins, |z| <= 3 {np.mean(z <= 3):.4f}, max {z.max():.2f}", flush=True)
    assert np.mean(z <= 3) >= 0.98
    assert z.max() < 5.0


def test_monopole_offset_is_the_third_order_term(ensemble):
    """The few-percent offset of B_0^0 from [B]_d at f_NG = 0.5 is the term
    third order in f_NG (a share of B growing as f_NG^2), not a first-order
    bias: the first-order part matches Bexact to well under a percent."""
    o = ensemble["orders"][12]
    j = ensemble["lms"].index((0, 0))
    ok = np.isfinite(o["bd1"][j])
    first = o["c1"][j][ok] / o["bexact1"][j][ok] - 1.0
    third = 0.25 * o["c3"][j][ok] / o["c1"][j][ok]
    zt = o["c3"][j][ok] / o["c3_sigma"][j][ok]
    assert abs(np.median(first)) < 0.003
    assert 0.01 < np.median(third) < 0.06
    assert np.mean(zt > 5) > 0.9  # significant in nearly every bin
    # at f_NG = 0.25 the offset from [B]_d shrinks with the third-order share
    fr5 = ensemble["stats"][(0.5, 12)]["frac"][j][ok]
    fr25 = ensemble["stats"][(0.25, 12)]["frac"][j][ok]
    hi = ensemble["stats"][(0.5, 12)]["sigma"][j][ok] < 0.02 * np.abs(ensemble["stats"][(0.5, 12)]["bd"][j][ok])
    assert hi.sum() >= 20
    assert np.median(fr25[hi]) < 0.6 * np.median(fr5[hi])
